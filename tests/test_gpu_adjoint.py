"""GPU adjoint step (setd_etd_adjoint_step) and the checkpointed
differentiable integration (paper_2310_07551_amd.autograd) against the
oracle's discrete adjoint on small grids (FP64, 1e-11 relative), and against
central finite differences of the GPU forward run on the 3D FitzHugh-Nagumo
128^3, 200-step workload (h = 1e-6)."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from tests.gpu_util import dev, rel_l2, say, torch
import workloads as wl

pytestmark = pytest.mark.gpu

import paper_2310_07551_amd as setd   # noqa: E402
from paper_2310_07551_amd import autograd as sad   # noqa: E402

TOL = 1e-11


def _flat(U):
    return np.concatenate([np.asarray(x).ravel(order="F") for x in U])


def _small(kind):
    if kind == "fhn3d":
        p = wl.fhn_3d(dims=(12, 10, 9))
        p.U0 = [0.3 * np.random.default_rng(5 + c).standard_normal(x.shape) for c, x in enumerate(p.U0)]
        return p, 6
    if kind == "schnak2d":
        p = wl.schnakenberg_2d(20, 17, tau=2e-3)
        p.U0 = [x + 0.05 * np.random.default_rng(3 + c).standard_normal(x.shape) for c, x in enumerate(p.U0)]
        return p, 5
    # dense (non-tridiagonal), non-symmetric matrices: exercises the transposes
    p = wl.schnakenberg_2d(14, 18, tau=2e-3)
    rng = np.random.default_rng(8)
    p.A = [[M + 5.0 * np.triu(rng.standard_normal(M.shape), 1) / M.shape[0] for M in Ac] for Ac in p.A]
    p.U0 = [x + 0.05 * rng.standard_normal(x.shape) for x in p.U0]
    return p, 4


@pytest.mark.parametrize("kind", ["fhn3d", "schnak2d", "dense"])
def test_adjoint_matches_oracle(kind):
    p, n = _small(kind)
    rng = np.random.default_rng(11)
    target = [x + 0.1 * rng.standard_normal(x.shape) for x in p.U0]
    L, U0bar, pbar, sig = oadj.loss_and_gradients(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)
    say("adjoint", kind, p.dims, n, "L", L)
    # GPU: forward states, then adjoint steps backwards through them (C-ABI level)
    T = torch()
    ctx = setd.Context(p.dims, [[dev(M) for M in Ac] for Ac in p.A], p.tau)
    u = T.from_numpy(_flat(p.U0)).cuda()
    states = [u.clone()]
    for _ in range(n):
        ctx.step(u, 1, p.g_kind, p.params)
        states.append(u.clone())
    ubar = states[-1] - T.from_numpy(_flat(target)).cuda()
    grad = T.zeros(len(p.params) + 2, dtype=T.float64, device="cuda")
    for k in range(n - 1, -1, -1):
        ctx.adjoint_step(states[k], ubar, p.g_kind, p.params, grad, sigma_mask=3)
    T.cuda.synchronize()
    e_u = rel_l2(ubar.cpu().numpy(), _flat(U0bar))
    g = grad.cpu().numpy()
    e_p = np.abs(g[:len(p.params)] - pbar) / np.maximum(np.abs(pbar), 1e-300)
    e_s = np.abs(g[len(p.params):] - sig) / np.abs(sig)
    say("  ubar rel_l2 %.2e  params %s  sigma %s" % (e_u, e_p, e_s))
    assert e_u < TOL
    assert np.all(np.abs(g[:len(p.params)] - pbar) <= TOL * np.max(np.abs(pbar)))
    assert np.all(e_s < TOL)


def test_autograd_checkpointed_matches_oracle():
    p, n = _small("fhn3d")
    n = 7
    rng = np.random.default_rng(12)
    target = [x + 0.1 * rng.standard_normal(x.shape) for x in p.U0]
    L, U0bar, pbar, sig = oadj.loss_and_gradients(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)
    T = torch()
    D = [[dev(wl.neumann_d2(m)) for m in p.dims] for _ in range(2)]
    diff = T.tensor([p.A[0][0][1, 1] / wl.neumann_d2(p.dims[0])[1, 1],
                     p.A[1][0][1, 1] / wl.neumann_d2(p.dims[0])[1, 1]], dtype=T.float64, requires_grad=True)
    params = T.tensor(p.params, dtype=T.float64, requires_grad=True)
    u0 = T.from_numpy(_flat(p.U0)).cuda().requires_grad_(True)
    uT = sad.integrate(u0, params, diff, dims=p.dims, D=D, g_kind=p.g_kind, tau=p.tau, nsteps=n, checkpoint=3)
    loss = 0.5 * ((uT - T.from_numpy(_flat(target)).cuda()) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - L) <= 1e-12 * L
    assert rel_l2(u0.grad.cpu().numpy(), _flat(U0bar)) < TOL
    gp = params.grad.numpy()
    assert np.all(np.abs(gp - pbar) <= TOL * np.max(np.abs(pbar)))
    # oracle sigma gradient = diff * dL/ddiff
    gd = diff.grad.numpy() * diff.detach().numpy()
    assert np.all(np.abs(gd - sig) <= TOL * np.abs(sig))


def test_fhn128_200_steps_gradients_vs_central_differences():
    """3D FitzHugh-Nagumo 128^3, 200 steps, L = 1/2 ||u(T) - u_target||^2 with
    u_target from eps = 0.55, a1 = 2.1; adjoint gradients (checkpoint every 20
    steps) against central differences of the GPU forward run.

    The u0 direction uses h = 1e-6.  For the parameters the loss (about 1.5e-6)
    changes by only ~1e-10 over h = 1e-6 while its evaluations carry an
    absolute rounding noise of a few 1e-15, so h = 1e-6 resolves eps and a1 to
    ~1e-4 and d_v not at all; they use the fourth-order central stencil with
    steps 1e-3 relative (measured: it agrees with the adjoint to 3e-8, 8e-8
    and 9e-6, and converges between 1e-5 and 3e-3; 1e-2 is already too wide
    for d_v), and the h = 1e-6 differences are printed beside them.  d_v's
    gradient is ~1e4 times smaller than eps's, so its difference carries a
    noise of ~5e-5 relative at this step; its tolerance is 1e-4."""
    T = torch()
    p = wl.make("fhn3d_128", nsteps=200)
    nsteps = 200
    D = [[dev(wl.neumann_d2(m)) for m in p.dims] for _ in range(2)]
    du, dv = 1.0, float(p.A[1][0][1, 1] / wl.neumann_d2(p.dims[0])[1, 1])
    eps, a1, a0 = p.params[:3]
    u0 = T.from_numpy(p.u0_flat()).cuda()

    def run(u_init, e, a, dvv):
        with T.no_grad():
            return sad.integrate(u_init, T.tensor([e, a, a0], dtype=T.float64), T.tensor([du, dvv], dtype=T.float64),
                                 dims=p.dims, D=D, g_kind=p.g_kind, tau=p.tau, nsteps=nsteps, checkpoint=nsteps)

    target = run(u0, 0.55, 2.1, dv).clone()

    def loss_of(u_init, e, a, dvv):
        return 0.5 * float(((run(u_init, e, a, dvv) - target) ** 2).sum().item())

    params = T.tensor([eps, a1, a0], dtype=T.float64, requires_grad=True)
    diff = T.tensor([du, dv], dtype=T.float64, requires_grad=True)
    ui = u0.clone().requires_grad_(True)
    uT = sad.integrate(ui, params, diff, dims=p.dims, D=D, g_kind=p.g_kind, tau=p.tau, nsteps=nsteps, checkpoint=20)
    loss = 0.5 * ((uT - target) ** 2).sum()
    loss.backward()
    L0 = loss_of(u0, eps, a1, dv)
    assert L0 == loss_of(u0, eps, a1, dv)          # the forward run is deterministic
    assert abs(L0 - loss.item()) <= 1e-12 * L0
    say("loss", L0)

    def fd2(f, x, h):
        return (f(x + h) - f(x - h)) / (2 * h)

    def fd4(f, x, h):
        return (8 * (f(x + h) - f(x - h)) - (f(x + 2 * h) - f(x - 2 * h))) / (12 * h)

    f_eps = lambda x: loss_of(u0, x, a1, dv)
    f_a1 = lambda x: loss_of(u0, eps, x, dv)
    f_dv = lambda x: loss_of(u0, eps, a1, x)
    dirn = T.from_numpy(np.random.default_rng(3).standard_normal(u0.numel())).cuda()
    f_u = lambda x: loss_of(u0 + x * dirn, eps, a1, dv)
    checks = [("eps", fd4(f_eps, eps, 1e-3 * eps), fd2(f_eps, eps, 1e-6), params.grad[0].item(), 1e-5),
              ("a1", fd4(f_a1, a1, 1e-3 * a1), fd2(f_a1, a1, 1e-6), params.grad[1].item(), 1e-5),
              ("dv", fd4(f_dv, dv, 1e-3 * dv), fd2(f_dv, dv, 1e-6), diff.grad[1].item(), 1e-4),
              ("u0 direction", fd2(f_u, 0.0, 1e-6), None, float((ui.grad * dirn).sum().item()), 1e-5)]
    for name, fd, fd_small, ad, tol in checks:
        say("  %-13s fd %.10e adjoint %.10e rel %.2e%s" % (
            name, fd, ad, abs(fd - ad) / abs(fd),
            "" if fd_small is None else "   (h = 1e-6: %.10e, rel %.2e)" % (fd_small, abs(fd_small - ad) / abs(ad))))
    for name, fd, fd_small, ad, tol in checks:
        assert abs(fd - ad) <= tol * abs(fd), name


@pytest.mark.parametrize("kind", ["fhn3d", "schnak2d", "dense"])
def test_recorded_step_and_adjoint(kind):
    """setd_etd_step_record: the same new state as setd_etd_step (bit for
    bit), stage quantities G, F, U2, D2, U3, D3 equal to the oracle's (eq.
    exprk3 with the split actions, composed here from the oracle's pieces),
    and setd_etd_adjoint_step_recorded gives the oracle's gradients."""
    import oracle
    p, n = _small(kind)
    T = torch()
    ctx = setd.Context(p.dims, [[dev(M) for M in Ac] for Ac in p.A], p.tau)
    N = int(np.prod(p.dims))
    u_rec = T.from_numpy(_flat(p.U0)).cuda()
    u_ref = u_rec.clone()
    states = [u_rec.clone()]
    recs = T.empty((n, 6 * 2 * N), dtype=T.float64, device="cuda")
    for k in range(n):
        ctx.step_record(u_rec, recs[k], p.g_kind, p.params)
        ctx.step(u_ref, 1, p.g_kind, p.params)
        states.append(u_rec.clone())
    T.cuda.synchronize()
    assert T.equal(u_rec, u_ref), (u_rec - u_ref).abs().max().item()
    # stage quantities of the first step against the oracle
    banks = oracle.make_banks(p.A, p.tau)
    U = p.U0
    G = oracle.reaction(p.g_kind, U, p.params)
    F = [oracle.kron_sum_action(U[c], p.A[c]) + G[c] for c in range(2)]
    U2 = [U[c] + p.tau / 3.0 * banks[c].split_apply(1, 2, F[c]) for c in range(2)]
    G2 = oracle.reaction(p.g_kind, U2, p.params)
    D2 = [G2[c] - G[c] for c in range(2)]
    U3 = [U[c] + 2.0 * p.tau / 3.0 * banks[c].split_apply(1, 3, F[c])
          + 4.0 * p.tau / 3.0 * banks[c].split_apply(2, 3, D2[c]) for c in range(2)]
    G3 = oracle.reaction(p.g_kind, U3, p.params)
    D3 = [G3[c] - G[c] for c in range(2)]
    r0 = recs[0].cpu().numpy()
    for q, (name, ref) in enumerate((("G", G), ("F", F), ("U2", U2), ("D2", D2), ("U3", U3), ("D3", D3))):
        got = r0[q * 2 * N:(q + 1) * 2 * N]
        e = rel_l2(got, _flat(ref))
        say("  rec %s rel_l2 %.2e" % (name, e))
        assert e < 1e-12, (name, e)
    # adjoint through the recorded stages against the oracle's gradients
    rng = np.random.default_rng(11)
    target = [x + 0.1 * rng.standard_normal(x.shape) for x in p.U0]
    L, U0bar, pbar, sig = oadj.loss_and_gradients(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)
    ubar = states[-1] - T.from_numpy(_flat(target)).cuda()
    grad = T.zeros(len(p.params) + 2, dtype=T.float64, device="cuda")
    for k in range(n - 1, -1, -1):
        ctx.adjoint_step(states[k], ubar, p.g_kind, p.params, grad, sigma_mask=3, rec=recs[k])
    T.cuda.synchronize()
    e_u = rel_l2(ubar.cpu().numpy(), _flat(U0bar))
    g = grad.cpu().numpy()
    say("  recorded adjoint: ubar rel_l2 %.2e" % e_u)
    assert e_u < TOL
    assert np.all(np.abs(g[:len(p.params)] - pbar) <= TOL * np.max(np.abs(pbar)))
    assert np.all(np.abs(g[len(p.params):] - sig) < TOL * np.abs(sig))


def test_autograd_without_recording_matches_oracle():
    """The checkpointed backward pass with record=False (the adjoint steps
    recompute their stages) gives the same gradients."""
    p, _ = _small("fhn3d")
    n = 5
    rng = np.random.default_rng(13)
    target = [x + 0.1 * rng.standard_normal(x.shape) for x in p.U0]
    L, U0bar, pbar, sig = oadj.loss_and_gradients(p.U0, p.A, p.tau, n, p.g_kind, p.params, target)
    T = torch()
    D = [[dev(wl.neumann_d2(m)) for m in p.dims] for _ in range(2)]
    diff = T.tensor([p.A[0][0][1, 1] / wl.neumann_d2(p.dims[0])[1, 1],
                     p.A[1][0][1, 1] / wl.neumann_d2(p.dims[0])[1, 1]], dtype=T.float64, requires_grad=True)
    params = T.tensor(p.params, dtype=T.float64, requires_grad=True)
    u0 = T.from_numpy(_flat(p.U0)).cuda().requires_grad_(True)
    uT = sad.integrate(u0, params, diff, dims=p.dims, D=D, g_kind=p.g_kind, tau=p.tau, nsteps=n, checkpoint=2,
                       record=False)
    loss = 0.5 * ((uT - T.from_numpy(_flat(target)).cuda()) ** 2).sum()
    loss.backward()
    assert rel_l2(u0.grad.cpu().numpy(), _flat(U0bar)) < TOL
    assert np.all(np.abs(params.grad.numpy() - pbar) <= TOL * np.max(np.abs(pbar)))
    gd = diff.grad.numpy() * diff.detach().numpy()
    assert np.all(np.abs(gd - sig) <= TOL * np.abs(sig))
