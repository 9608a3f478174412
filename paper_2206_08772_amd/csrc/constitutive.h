// Constitutive building blocks shared by the forward material-point pass and
// its adjoint: material constants in the working precision, the flow stress
// (Johnson-Cook, Sec. 4.2; linear hardening, Sec. 4.1) and the scalar
// return-map Newton solve.
#pragma once

#include "otm_common.h"

namespace otm {

// ----------------------------------------------------------- scalar math
OTM_DEV double m_log1p(double v) { return log1p(v); }
OTM_DEV float m_log1p(float v) { return log1pf(v); }
OTM_DEV double m_expm1(double v) { return expm1(v); }
OTM_DEV float m_expm1(float v) { return expm1f(v); }
OTM_DEV double m_log(double v) { return log(v); }
OTM_DEV float m_log(float v) { return logf(v); }
// a^b for a > 0 (every caller guards it) as exp(b log a): the relative error
// is about (2 + |b log a|) ulp, far below the float64 tolerance for the
// strains and homologous temperatures of the flow law, and it needs far fewer
// registers than the library pow, whose extended-precision log would set the
// register peak of the material-point pass.
OTM_DEV double m_pow(double a, double b) { return exp(b * log(a)); }
OTM_DEV float m_pow(float a, float b) { return powf(a, b); }
OTM_DEV double m_sqrt(double v) { return sqrt(v); }
OTM_DEV float m_sqrt(float v) { return sqrtf(v); }

// Material constants in the working precision.
template <typename R>
struct Mat {
  int model;
  R K, mu, lamL;
  R A, B, n, C, m, rate0dt, Tr, Tm, rhoCp, chi, Y0, H;
  R tol;
  int max_iter;
  double jd[5];      // Johnson-Cook fracture constants d1..d5 (float64)
  double rate0dt_d;  // dt * eps_dot0 in float64 (fracture rate term)
};

// Thermal softening factor 1 - T*^m of the Johnson-Cook law (1 below T_r).
template <typename R>
OTM_DEV R thermal_factor(const Mat<R>& M, R Ts) {
  return Ts > R(0) ? R(1) - m_pow(Ts, M.m) : R(1);
}

// sigma_Y(eb + x, x / dt, T*) and its derivative in x, with the thermal
// factor of T* given (it does not change during a return-map solve).
template <typename R>
OTM_DEV void flow_stress_t(const Mat<R>& M, R eb, R x, R therm, R& sy, R& dsy) {
  if (M.model == OTM_J2_LINEAR) {
    sy = M.Y0 + M.H * (eb + x);
    dsy = M.H;
    return;
  }
  const R e = eb + x;
  R hard = M.A, dhard = R(INFINITY);
  if (e > R(0)) {
    const R en = m_pow(e, M.n);
    hard = M.A + M.B * en;
    dhard = M.B * M.n * en / e;
  }
  const R ratio = x / M.rate0dt;
  R rate = R(1), drate = R(0);
  if (ratio > R(1)) {
    rate = R(1) + M.C * m_log(ratio);
    drate = M.C / x;
  }
  sy = hard * rate * therm;
  dsy = (dhard * rate + hard * drate) * therm;
}

template <typename R>
OTM_DEV void flow_stress(const Mat<R>& M, R eb, R x, R Ts, R& sy, R& dsy) {
  flow_stress_t(M, eb, x, thermal_factor(M, Ts), sy, dsy);
}

// Root of q - 3 mu x - sigma_Y(eb + x, x/dt, T*) on (0, (q - sigma_Y0)/(3 mu)]:
// Newton from the right end, bracket kept on the sign, bisection when the
// Newton iterate leaves the bracket.  Stops when the residual is at the
// rounding level (|g| <= tol q; the only test that can end the iteration for
// MPs that barely yield) or the step or bracket is below tol of the iterate.
template <typename R>
OTM_DEV R solve_return(const Mat<R>& M, R q, R eb, R Ts, R sy0, bool& ok) {
  const R therm = thermal_factor(M, Ts);
  R x = (q - sy0) / (R(3) * M.mu);
  R lo = R(0), hi = x;
  ok = false;
  for (int it = 0; it < M.max_iter; ++it) {
    R sy, dsy;
    flow_stress_t(M, eb, x, therm, sy, dsy);
    const R g = q - R(3) * M.mu * x - sy;
    if (fabs(g) <= M.tol * q) { ok = true; break; }
    const R gp = -R(3) * M.mu - dsy;
    if (g > R(0)) lo = x; else hi = x;
    R xn = x - g / gp;
    if (!(xn > lo && xn < hi)) xn = R(0.5) * (lo + hi);
    const bool small = fabs(xn - x) <= M.tol * fabs(xn) || (hi - lo) <= M.tol * hi;
    x = xn;
    if (small) { ok = true; break; }
  }
  return x;
}

template <typename R>
inline Mat<R> make_mat(const otm_params& p, double dt) {
  Mat<R> M;
  const double lamL = p.E * p.nu / ((1 + p.nu) * (1 - 2 * p.nu));
  const double mu = p.E / (2 * (1 + p.nu));
  M.model = p.model;
  M.K = (R)(lamL + 2.0 * mu / 3.0);
  M.mu = (R)mu;
  M.lamL = (R)lamL;
  M.A = (R)p.A; M.B = (R)p.B; M.n = (R)p.n; M.C = (R)p.C; M.m = (R)p.m;
  M.rate0dt = (R)(dt * p.eps_dot0);
  M.Tr = (R)p.T_r; M.Tm = (R)p.T_m;
  M.rhoCp = (R)(p.rho0 * p.Cp);
  M.chi = (R)p.chi;
  M.Y0 = (R)p.Y0; M.H = (R)p.H;
  const double eps = sizeof(R) == 8 ? 2.2e-16 : 1.2e-7;
  M.tol = (R)(p.rm_tol > 4 * eps ? p.rm_tol : 4 * eps);
  M.max_iter = p.rm_max_iter;
  for (int k = 0; k < 5; ++k) M.jd[k] = p.jc_d[k];
  M.rate0dt_d = dt * p.eps_dot0;
  return M;
}

}  // namespace otm
