// Directional-splitting coefficients of exprk3ds_real.
//
// d = 2: the two-term splitting eq. (split2d) with l_1 = 1, l_2 = 2 and the
//        real solutions of Table 1 (direction-dependent alpha).
// d > 2: the three-term splitting eq. (splitnd3) with l_1 = l_3 = 1, l_2 = 2
//        and Table 3 (alpha the same in every direction, eta_2 ~ 2^{d-3}).
// Section 2.4: the '+' sign of alpha_{1,1} (alpha_{1,mu}) is used, and the
// upper signs of a column belong together.
#pragma once

#include <cmath>

namespace setd {

struct Splitting {
  int nterms;
  int ell_i[3];        // phi index of each term
  double eta[3];
  double alpha[3][3];  // [term][direction]
};

// phi_ell, ell in {1, 2}, dimension d in {2, 3, ...}.
inline Splitting splitting(int ell, int d) {
  Splitting S{};
  if (d == 2) {
    S.nterms = 2;
    S.ell_i[0] = 1;
    S.ell_i[1] = 2;
    if (ell == 1) {
      const double q = std::sqrt(10.0);
      S.eta[0] = -1.25;
      S.eta[1] = 9.0;
      S.alpha[0][0] = 4.0 / 3.0 + 4.0 * q / 15.0;
      S.alpha[0][1] = 4.0 / 3.0 - 4.0 * q / 15.0;
      S.alpha[1][0] = 16.0 / 9.0 + 2.0 * q / 9.0;
      S.alpha[1][1] = 16.0 / 9.0 - 2.0 * q / 9.0;
    } else {
      const double q = std::sqrt(33.0);
      S.eta[0] = -4.0 / 3.0;
      S.eta[1] = 22.0 / 3.0;
      S.alpha[0][0] = 9.0 / 8.0 + q / 8.0;
      S.alpha[0][1] = 9.0 / 8.0 - q / 8.0;
      S.alpha[1][0] = 1.5 + 3.0 * q / 22.0;
      S.alpha[1][1] = 1.5 - 3.0 * q / 22.0;
    }
    return S;
  }
  S.nterms = 3;
  S.ell_i[0] = 1;
  S.ell_i[1] = 2;
  S.ell_i[2] = 1;
  const double pw = std::ldexp(1.0, d - 3);
  double a1, a2, a3;
  if (ell == 1) {
    const double q = std::sqrt(2991111.0);
    S.eta[0] = 2243.0 / 1350.0 + 440521.0 / (675.0 * q);
    S.eta[1] = -12544.0 / 675.0 * pw;
    S.eta[2] = 2243.0 / 1350.0 - 440521.0 / (675.0 * q);
    a1 = 3.0 * (5161.0 + q) / 15869.0;
    a2 = 45.0 / 28.0;
    a3 = 3.0 * (5161.0 - q) / 15869.0;
  } else {
    const double q = std::sqrt(2391.0);
    S.eta[0] = 19.0 / 27.0 + 151.0 / (27.0 * q);
    S.eta[1] = -196.0 / 27.0 * pw;
    S.eta[2] = 19.0 / 27.0 - 151.0 / (27.0 * q);
    a1 = 3.0 * (121.0 + q) / 490.0;
    a2 = 9.0 / 7.0;
    a3 = 3.0 * (121.0 - q) / 490.0;
  }
  for (int mu = 0; mu < 3; ++mu) {
    S.alpha[0][mu] = a1;
    S.alpha[1][mu] = a2;
    S.alpha[2][mu] = a3;
  }
  return S;
}

// Two-term splitting with complex coefficients (exprk3ds_cplx): the complex
// column of Table 1 for d = 2 and Table 2 for d > 2 (which reduces to it at
// d = 2), upper signs; ell_i = (1, 2); alpha is the same in every direction.
// The conjugate set gives the same real part of every split action.
struct SplittingC {
  double eta_r[2], eta_i[2];
  double al_r[2], al_i[2];
};

inline SplittingC splitting_cplx(int ell, int d) {
  SplittingC S{};
  const double pw = std::ldexp(1.0, d - 2);
  if (ell == 1) {
    const double q = std::sqrt(2.0);
    S.eta_r[0] = 7.0 / 4.0;
    S.eta_i[0] = 1.5 * q;
    S.eta_r[1] = -3.0 * pw;
    S.eta_i[1] = -6.0 * q * pw;
    S.al_r[0] = 12.0 / 11.0;
    S.al_i[0] = -4.0 * q / 11.0;
    S.al_r[1] = 4.0 / 3.0;
    S.al_i[1] = -2.0 * q / 3.0;
  } else {
    const double q = std::sqrt(3.0);
    S.eta_r[0] = 2.0 / 3.0;
    S.eta_i[0] = 2.0 * q / 3.0;
    S.eta_r[1] = -2.0 / 3.0 * pw;
    S.eta_i[1] = -8.0 * q / 3.0 * pw;
    S.al_r[0] = 0.75;
    S.al_i[0] = -q / 4.0;
    S.al_r[1] = 6.0 / 7.0;
    S.al_i[1] = -3.0 * q / 7.0;
  }
  return S;
}

// Argument scale c_s of the stages of eq. exprk3.
inline double stage_scale(int stage) {
  return stage == 2 ? 1.0 / 3.0 : (stage == 3 ? 2.0 / 3.0 : 1.0);
}

}  // namespace setd
