// Adjoint (reverse-mode derivative) of one explicit step, float64.
//
// Given the adjoint of the state after step n (bar_next) and the stored
// forward states n and n+1 (tapes), it produces the adjoint of state n and
// adds the step's contribution to the gradient with respect to the hardening
// constants.  Support lists are those of the stored trajectory (frozen).  The
// step's data flow, reversed:
//
//   K1  shape functions of state n+1 (LME, Sec. 2.3): N_I = softmax(f_I),
//       f_I = -beta |d_I|^2 + lambda . d_I, grad N_I = -N_I J^{-1} d_I, with
//       lambda(d) implicit through sum N_I d_I = 0.  From the adjoints of N and
//       grad N per pair it forms the adjoint of each offset d_I = x_p - x_I:
//       x_p gets the sum, node I the negative (pre-summed in LDS, then
//       float64 atomics).
//   K3  MP update: x_p' = sum N_I x_I', dF = 1 + sum du_I' (x) grad N_I,
//       F' = dF F, v' = det(dF) v and the J2 return map (Sec. 4.1/4.2) with
//       Hencky strain: the spectral derivative of the isotropic tensor
//       functions b_tr -> tau, b^e' (divided differences, stable for equal
//       eigenvalues), the scalar chain through q_tr, and the implicit
//       derivative of the return equation for dEpsbar, which also gives the
//       parameter gradient.  Node adjoints of x' and du' are pre-summed in LDS.
//   K5  node update (central difference + wall projection).
//   K6  lumped mass and force of state n (nodal mass / residual equations).
#include "constitutive.h"
#include "launch.h"
#include "otm_common.h"

namespace otm {

// ------------------------------------------------------------------ helpers
// Workgroup-level sum of NV node values per node id in an LDS hash table,
// flushed to global memory with one float64 atomic per node and value.
template <int NV, int BITS>
struct NodeSums {
  static constexpr int kSlots = 1 << BITS;
  int32_t keys[kSlots];
  double vals[NV][kSlots];
};

template <int NV, int BITS>
OTM_DEV void sums_clear(NodeSums<NV, BITS>& t) {
  for (int s = threadIdx.x; s < NodeSums<NV, BITS>::kSlots; s += blockDim.x) {
    t.keys[s] = -1;
#pragma unroll
    for (int v = 0; v < NV; ++v) t.vals[v][s] = 0.0;
  }
}

// dst[v] is the v-th destination array ([n] each); values go to dst[v][I].
template <int NV, int BITS>
OTM_DEV void sums_add(NodeSums<NV, BITS>& t, int32_t I, const double c[NV],
                      double* const dst[NV]) {
  constexpr int kSlots = NodeSums<NV, BITS>::kSlots;
  uint32_t h = ((uint32_t)I * 2654435761u) >> (32 - BITS);
  for (int probe = 0; probe < 32; ++probe) {
    const int32_t prev = atomicCAS(&t.keys[h], -1, I);
    if (prev == -1 || prev == I) {
#pragma unroll
      for (int v = 0; v < NV; ++v) atomicAdd(&t.vals[v][h], c[v]);
      return;
    }
    h = (h + 1) & (kSlots - 1);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) atomicAdd(&dst[v][I], c[v]);  // crowded table
}

template <int NV, int BITS>
OTM_DEV void sums_flush(NodeSums<NV, BITS>& t, double* const dst[NV]) {
  for (int s = threadIdx.x; s < NodeSums<NV, BITS>::kSlots; s += blockDim.x) {
    const int32_t I = t.keys[s];
    if (I < 0) continue;
#pragma unroll
    for (int v = 0; v < NV; ++v) atomicAdd(&dst[v][I], t.vals[v][s]);
  }
}

OTM_HD void mat3_mul(const double A[3][3], const double B[3][3], double C[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i][j] = A[i][0] * B[0][j] + A[i][1] * B[1][j] + A[i][2] * B[2][j];
}
// cof(A) = det(A) A^{-T}
OTM_HD void cofactor3(const double A[3][3], double C[3][3]) {
  C[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  C[0][1] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  C[0][2] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  C[1][0] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
  C[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
  C[1][2] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
  C[2][0] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
  C[2][1] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
  C[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
}
OTM_HD double det3m(const double A[3][3]) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
         A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

constexpr int kVi[6] = {0, 1, 2, 0, 1, 0}, kVj[6] = {0, 1, 2, 1, 2, 2};

// Adjoint of the 6 stored components of a symmetric tensor -> the symmetric
// full-matrix adjoint (dL = sum_ij Sb_ij dS_ij), and back.
OTM_HD void voigt_bar_to_full(const double v[6], double S[3][3]) {
  for (int c = 0; c < 6; ++c) {
    const double w = c < 3 ? v[c] : 0.5 * v[c];
    S[kVi[c]][kVj[c]] = w;
    S[kVj[c]][kVi[c]] = w;
  }
}
OTM_HD void full_bar_to_voigt(const double S[3][3], double v[6]) {
  for (int c = 0; c < 6; ++c)
    v[c] = c < 3 ? S[c][c] : S[kVi[c]][kVj[c]] + S[kVj[c]][kVi[c]];
}

// u / expm1(u) and expm1(a u) / expm1(u), accurate near u = 0.
OTM_HD double ratio_u_expm1(double u) {
  return fabs(u) < 1e-8 ? 1.0 - 0.5 * u : u / expm1(u);
}
OTM_HD double ratio_expm1(double a, double u) {
  return fabs(u) < 1e-8 ? a * (1.0 + 0.5 * (a - 1.0) * u) : expm1(a * u) / expm1(u);
}

// Partial derivatives of the flow stress at (eb + x, x/dt, T*): by epsbar,
// by T* and by the kTheta hardening constants (A, B, n, C, m of Johnson-Cook;
// Y0, H of linear hardening, the other three 0).
constexpr int kTheta = 5;
struct FlowPartials {
  double s_eb, s_T, s_th[kTheta];
};
OTM_DEV FlowPartials flow_partials(const Mat<double>& M, double eb, double x, double Ts) {
  FlowPartials P{0.0, 0.0, {0.0, 0.0, 0.0, 0.0, 0.0}};
  if (M.model == OTM_J2_LINEAR) {
    P.s_eb = M.H;
    P.s_th[0] = 1.0;       // d/dY0
    P.s_th[1] = eb + x;    // d/dH
    return P;
  }
  const double e = eb + x;
  double en = 0.0, hard = M.A, dhard = 0.0, lne = 0.0;
  if (e > 0.0) {
    lne = log(e);
    en = exp(M.n * lne);  // e^n, as in the forward flow law
    hard = M.A + M.B * en;
    dhard = M.B * M.n * en / e;
  }
  const double ratio = x / M.rate0dt;
  const double lrate = ratio > 1.0 ? log(ratio) : 0.0;
  const double rate = 1.0 + M.C * lrate;
  double therm = 1.0, dtherm = 0.0, dtherm_m = 0.0;
  if (Ts > 0.0) {
    const double tm = m_pow(Ts, M.m);
    therm = 1.0 - tm;
    dtherm = -M.m * tm / Ts;
    dtherm_m = -tm * log(Ts);
  }
  P.s_eb = dhard * rate * therm;
  P.s_T = hard * rate * dtherm;
  P.s_th[0] = rate * therm;                 // d/dA
  P.s_th[1] = en * rate * therm;            // d/dB
  P.s_th[2] = M.B * en * lne * rate * therm;  // d/dn
  P.s_th[3] = hard * lrate * therm;         // d/dC
  P.s_th[4] = hard * rate * dtherm_m;       // d/dm
  return P;
}

// ---------------------------------------------------------------- K1: LME
// Supports of up to 40 nodes take 8 lanes with 5 pairs each (one launch);
// the rare longer ones, up to 48, a second launch with 16 lanes x 3 pairs.
constexpr int kAdjG = 8, kAdjPPL = 5;
constexpr int kAdjLongG = 16, kAdjLongPPL = 3;
static_assert(kAdjLongG * kAdjLongPPL == 48, "the documented adjoint support limit");
constexpr int kAdjLmeRounds = 8;  // MPs per workgroup = (256 / G) * rounds

struct AdjLmeArgs {
  int64_t n_nodes, n_mp, stride;
  const double4* nrec;   // node records of state n+1: 2 I = (x, y, z, du_x)
  const double* xp;      // [3][n_mp]
  const double* lam;     // [3][n_mp]
  const int64_t* off;
  const int32_t* idx;
  const double* Nb;      // adjoint of N per pair
  const double* dNb;     // adjoint of grad N per pair [3][stride]
  double beta;
  double* xpb;           // out: adjoint of x_p from the shape functions [3][n_mp]
  double* xb;            // in/out: adjoint of node positions [3][n_nodes]
  otm_diag* diag;
};

// Handles the MPs with KMIN < K <= G * PPL support nodes; the launch with
// KMIN = 0 also writes the zero adjoint of empty supports, the one with LAST
// that of over-long supports, which it reports.
template <int G, int PPL, int KMIN, bool LAST>
__global__ __launch_bounds__(256) void k_adj_lme(AdjLmeArgs a) {
  __shared__ NodeSums<3, 10> tab;
  if constexpr (KMIN > 0) {
    // workgroups without a support longer than KMIN leave at once
    bool any = false;
    for (int round = 0; round < kAdjLmeRounds; ++round) {
      const int64_t p = ((int64_t)xcd_block() * kAdjLmeRounds + round) * (256 / G) + threadIdx.x / G;
      if (p < a.n_mp && threadIdx.x % G == 0) any |= a.off[p + 1] - a.off[p] > KMIN;
    }
    if (!__syncthreads_or(any)) return;
  }
  sums_clear(tab);
  __syncthreads();
  double* const dst[3] = {a.xb, a.xb + a.n_nodes, a.xb + 2 * a.n_nodes};
  const int lane = threadIdx.x % G;
  for (int round = 0; round < kAdjLmeRounds; ++round) {
    const int64_t p = ((int64_t)xcd_block() * kAdjLmeRounds + round) * (256 / G) + threadIdx.x / G;
    if (p >= a.n_mp) continue;
    const int64_t o = a.off[p];
    const int K = (int)(a.off[p + 1] - o);
    if (K <= KMIN || K > G * PPL) {
      if (lane == 0 && ((KMIN == 0 && K == 0) || (LAST && K > G * PPL))) {
        a.xpb[p] = a.xpb[a.n_mp + p] = a.xpb[2 * a.n_mp + p] = 0.0;
        if (K > 0) diag_fail(a.diag, OTM_ERR_SUPPORT, (uint64_t)p);
      }
      continue;
    }
    const double px = a.xp[p], py = a.xp[a.n_mp + p], pz = a.xp[2 * a.n_mp + p];
    const double lam[3] = {a.lam[p], a.lam[a.n_mp + p], a.lam[2 * a.n_mp + p]};
    double d[PPL][3], e[PPL], Nb[PPL], Gb[PPL][3];
    int32_t node[PPL];
    bool use[PPL];
    double fm = -INFINITY;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int q = k * G + lane;
      use[k] = q < K;
      const int64_t qq = o + (use[k] ? q : 0);
      node[k] = a.idx[qq];
      const double4 xI = a.nrec[2 * (int64_t)node[k]];
      d[k][0] = px - xI.x;
      d[k][1] = py - xI.y;
      d[k][2] = pz - xI.z;
      Nb[k] = a.Nb[qq];
      Gb[k][0] = a.dNb[qq];
      Gb[k][1] = a.dNb[a.stride + qq];
      Gb[k][2] = a.dNb[2 * a.stride + qq];
      const double prior = -a.beta * ((d[k][0] * d[k][0] + d[k][1] * d[k][1]) + d[k][2] * d[k][2]);
      e[k] = prior + (lam[0] * d[k][0] + lam[1] * d[k][1] + lam[2] * d[k][2]);
      if (use[k]) fm = fmax(fm, e[k]);
    }
    fm = group_max<G>(fm);
    // forward quantities at the stored multiplier
    double Z = 0, r[3] = {0, 0, 0}, S[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      e[k] = use[k] ? exp(e[k] - fm) : 0.0;
      Z += e[k];
      for (int i = 0; i < 3; ++i) r[i] += e[k] * d[k][i];
      for (int c = 0; c < 6; ++c) S[c] += e[k] * d[k][kVi[c]] * d[k][kVj[c]];
    }
    Z = group_sum<G>(Z);
    for (int i = 0; i < 3; ++i) r[i] = group_sum<G>(r[i]);
    for (int c = 0; c < 6; ++c) S[c] = group_sum<G>(S[c]);
    const double iz = 1.0 / Z;
    for (int i = 0; i < 3; ++i) r[i] *= iz;
    double J[6], Mi[6], det;
    for (int c = 0; c < 6; ++c) J[c] = S[c] * iz - r[kVi[c]] * r[kVj[c]];
    sym_inv(J, Mi, det);
    double Nq[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) Nq[k] = e[k] * iz;

    // grad N_I = -N_I M d_I
    double db[PPL][3], Mb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      double Md[3], MG[3];
      sym_mul_vec(Mi, d[k], Md);
      sym_mul_vec(Mi, Gb[k], MG);
      Nb[k] -= Gb[k][0] * Md[0] + Gb[k][1] * Md[1] + Gb[k][2] * Md[2];
      for (int i = 0; i < 3; ++i) db[k][i] = -Nq[k] * MG[i];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Mb[i][j] -= Nq[k] * Gb[k][i] * d[k][j];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Mb[i][j] = group_sum<G>(Mb[i][j]);
    // M = J^{-1}:  Jb = -M Mb M
    double Mf[3][3], T1[3][3], Jb[3][3];
    for (int c = 0; c < 6; ++c) { Mf[kVi[c]][kVj[c]] = Mi[c]; Mf[kVj[c]][kVi[c]] = Mi[c]; }
    mat3_mul(Mf, Mb, T1);
    mat3_mul(T1, Mf, Jb);
    double Js[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Js[i][j] = -(Jb[i][j] + Jb[j][i]);  // adjoint of sym part
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Jb[i][j] = -Jb[i][j];
    // J = sum N d d^T - r r^T,  r = sum N d
    double rb[3];
    for (int i = 0; i < 3; ++i) rb[i] = -(Js[i][0] * r[0] + Js[i][1] * r[1] + Js[i][2] * r[2]);
    double s1 = 0.0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      double Jd[3], dJd = 0.0;
      for (int i = 0; i < 3; ++i) {
        Jd[i] = Js[i][0] * d[k][0] + Js[i][1] * d[k][1] + Js[i][2] * d[k][2];
        for (int j = 0; j < 3; ++j) dJd += d[k][i] * Jb[i][j] * d[k][j];
      }
      Nb[k] += dJd + rb[0] * d[k][0] + rb[1] * d[k][1] + rb[2] * d[k][2];
      for (int i = 0; i < 3; ++i) db[k][i] += Nq[k] * (Jd[i] + rb[i]);
      s1 += use[k] ? Nq[k] * Nb[k] : 0.0;
    }
    s1 = group_sum<G>(s1);
    // N = softmax(f), f = -beta |d|^2 + lambda . d
    double lb[3] = {0, 0, 0}, gk[PPL][3];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const double fb = use[k] ? Nq[k] * (Nb[k] - s1) : 0.0;
      for (int i = 0; i < 3; ++i) {
        gk[k][i] = -2.0 * a.beta * d[k][i] + lam[i];
        db[k][i] += fb * gk[k][i];
        lb[i] += fb * d[k][i];
      }
    }
    for (int i = 0; i < 3; ++i) lb[i] = group_sum<G>(lb[i]);
    // lambda(d) from r(lambda, d) = 0: d_bar -= (dr/dd)^T J^{-1} lambda_bar
    double w[3];
    sym_mul_vec(Mi, lb, w);
    double xpb[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const double dw = (d[k][0] - r[0]) * w[0] + (d[k][1] - r[1]) * w[1] + (d[k][2] - r[2]) * w[2];
      for (int i = 0; i < 3; ++i) {
        db[k][i] -= Nq[k] * (w[i] + dw * gk[k][i]);
        if (use[k]) xpb[i] += db[k][i];
      }
    }
    for (int i = 0; i < 3; ++i) xpb[i] = group_sum<G>(xpb[i]);
    if (lane == 0) {
      a.xpb[p] = xpb[0];
      a.xpb[a.n_mp + p] = xpb[1];
      a.xpb[2 * a.n_mp + p] = xpb[2];
    }
    // d = x_p - x_I: node I gets -d_bar
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      if (!use[k]) continue;
      const double c[3] = {-db[k][0], -db[k][1], -db[k][2]};
      sums_add(tab, node[k], c, dst);
    }
  }
  __syncthreads();
  sums_flush(tab, dst);
}

// ------------------------------------------------ K3: MP update (J2 model)
constexpr int kAdjMpBlock = 128;
constexpr int kAdjGather = 8;
constexpr int kAdjGatherSlots = 4;

struct AdjMpArgs {
  int64_t n_nodes, n_mp, stride;  // stride: pair arrays of state n
  // state n (tape)
  const int64_t* off;
  const int32_t* idx;
  const double* N;
  const double* dN;
  const double* vol;
  const double* Fd;
  const double* bed;
  const double* epsbar;
  const double* T;
  // node records of state n+1: 2 I = (x, y, z, du_x), 2 I + 1 = (du_y, du_z, 0, 0)
  const double4* nrec;
  // adjoints of state n+1 (in)
  const double* xpb1;   // from K1
  const double* volb1;
  const double* Fdb1;
  const double* bedb1;
  const double* epsb1;
  const double* Tb1;
  const double* sigb1;
  // adjoints of state n (out)
  double* volb;
  double* Fdb;
  double* bedb;
  double* epsb;
  double* Tb;
  double* dfb;     // adjoint of dF per MP [9][n_mp] (written, workspace)
  double* theta_part;  // [gridDim][kTheta]
  Mat<double> M;
  double dt;
  otm_diag* diag;
};

// Adjoint of the MP update at MP p after the gather: dF = 1 + H of the step.
// Writes the adjoints of F_n, b^e_n, epsbar_n, T_n and v_n, adds the
// parameter-gradient terms to th and returns the adjoint of dF in dFb.
//
// The work runs in stages (forward recomputation; sigma and b^e'; scalar
// chain; the eigen-basis adjoint back to dF and b^e_n; F' = dF F_n), each
// loading its inputs where it starts and storing its outputs where they are
// final, with scheduling barriers between them, so that the live set stays
// within the 256 architectural VGPRs.  Spilling to AGPRs here is not safe:
// the compiler has been seen to place such spill copies ahead of the exec
// restore at the end of a divergent branch, leaving stale values in the lanes
// that skipped the branch.
OTM_DEV void mp_adjoint(const AdjMpArgs& a, int64_t p, const double dF[3][3], double dFb[3][3],
                        double thb[kTheta], bool& ok) {
  const Mat<double>& M = a.M;
  const int64_t n = a.n_mp;
  // ---- stage 1: forward recomputation (the same arithmetic as the MP pass)
  double d[3], V[3][3], e[3], dev[3], tr, q, Ts = 0.0, tunc = 0.0, deps = 0.0, c = 0.0;
  bool plastic;
  const double ebn = a.epsbar[p], Tn = a.T[p];
  {
    M3<double> h;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) h.a[i][j] = dF[i][j] - (i == j ? 1.0 : 0.0);
    S3<double> bds;
    for (int k = 0; k < 6; ++k) bds.v[k] = a.bed[k * n + p];
    const M3<double> B = full(bds);
    M3<double> HB;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        HB.a[i][j] = B.a[i][j] + h.a[i][0] * B.a[0][j] + h.a[i][1] * B.a[1][j] + h.a[i][2] * B.a[2][j];
    S3<double> dtr;
    for (int k = 0; k < 6; ++k) {
      const int i = kVi[k], j = kVj[k];
      const double hbh = HB.a[i][j] + HB.a[i][0] * h.a[j][0] + HB.a[i][1] * h.a[j][1] + HB.a[i][2] * h.a[j][2];
      dtr.v[k] = h.a[i][j] + h.a[j][i] +
                 (h.a[i][0] * h.a[j][0] + h.a[i][1] * h.a[j][1] + h.a[i][2] * h.a[j][2]) + hbh;
    }
    jacobi_eig(dtr, d, V);
  }
  for (int k = 0; k < 3; ++k) e[k] = 0.5 * log1p(d[k]);
  tr = e[0] + e[1] + e[2];
  for (int k = 0; k < 3; ++k) dev[k] = e[k] - tr / 3.0;
  q = 2.0 * M.mu * sqrt(1.5 * (dev[0] * dev[0] + dev[1] * dev[1] + dev[2] * dev[2]));
  if (M.model == OTM_J2_JC) {
    tunc = (Tn - M.Tr) / (M.Tm - M.Tr);
    Ts = tunc < 0.0 ? 0.0 : (tunc > 1.0 ? 1.0 : tunc);
  }
  {
    double sy0, dsy0;
    flow_stress(M, ebn, 0.0, Ts, sy0, dsy0);
    plastic = q > sy0;
    ok = true;
    if (plastic) {
      deps = solve_return(M, q, ebn, Ts, sy0, ok);
      c = 3.0 * M.mu * deps / q;
    }
  }
  double tau[3], bm1[3];
  for (int k = 0; k < 3; ++k) {
    tau[k] = M.K * tr + 2.0 * M.mu * (1.0 - c) * dev[k];
    bm1[k] = expm1(2.0 * (e[k] - c * dev[k]));
  }
  // derivative of the return equation in x and the flow-law partials at the
  // solution (plastic MPs), and the divided differences of tau_a and bm1_a
  // for the off-diagonal eigen-basis terms: all scalars, computed here while
  // few values are live
  double gx = 1.0;
  FlowPartials P{0.0, 0.0, {0.0, 0.0, 0.0}};
  if (plastic) {
    double sy, dsy;
    flow_stress(M, ebn, deps, Ts, sy, dsy);
    gx = -3.0 * M.mu - dsy;
    P = flow_partials(M, ebn, deps, Ts);
  }
  double rt[3], rbm[3];  // pairs (0,1), (1,2), (0,2)
  for (int k = 3; k < 6; ++k) {
    const int aa = kVi[k], bb = kVj[k];
    const double u = 2.0 * (e[aa] - e[bb]);
    rt[k - 3] = M.mu * (1.0 - c) * ratio_u_expm1(u) / (1.0 + d[bb]);
    rbm[k - 3] = (bm1[bb] + 1.0) * ratio_expm1(1.0 - c, u) / (1.0 + d[bb]);
  }
  double Jp;
  {
    double Fn[3][3], Fp[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Fn[i][j] = a.Fd[(3 * i + j) * n + p] + (i == j ? 1.0 : 0.0);
    mat3_mul(dF, Fn, Fp);
    Jp = det3m(Fp);
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage 2: sigma = V diag(tau) V^T / J', b^e' = 1 + V diag(bm1) V^T;
  // output adjoints in the eigen-basis (symmetric: xx yy zz xy yz xz)
  double Tt[6], Bt[6], Jpb;
  {
    double vb[6], Sb[3][3], Bb[3][3];
    for (int k = 0; k < 6; ++k) vb[k] = a.sigb1[k * n + p];
    voigt_bar_to_full(vb, Sb);
    for (int k = 0; k < 6; ++k) vb[k] = a.bedb1[k * n + p];
    voigt_bar_to_full(vb, Bb);
    // Tt = V^T (Sb / J') V and Bt = V^T Bb V; sigma : Sb = sum_a tau_a Tt_aa
    const double iJ = 1.0 / Jp;
    for (int bb = 0; bb < 3; ++bb) {
      double ws[3], wb[3];
      for (int i = 0; i < 3; ++i) {
        ws[i] = (Sb[i][0] * V[0][bb] + Sb[i][1] * V[1][bb] + Sb[i][2] * V[2][bb]) * iJ;
        wb[i] = Bb[i][0] * V[0][bb] + Bb[i][1] * V[1][bb] + Bb[i][2] * V[2][bb];
      }
      for (int aa = 0; aa <= bb; ++aa) {
        const int k = aa == bb ? aa : (aa == 0 ? (bb == 1 ? 3 : 5) : 4);
        Tt[k] = V[0][aa] * ws[0] + V[1][aa] * ws[1] + V[2][aa] * ws[2];
        Bt[k] = V[0][aa] * wb[0] + V[1][aa] * wb[1] + V[2][aa] * wb[2];
      }
    }
    Jpb = -(tau[0] * Tt[0] + tau[1] * Tt[1] + tau[2] * Tt[2]) * iJ;
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage 3: scalar chain through the principal values
  double Dt[6];
  {
    const double epsb1 = a.epsb1[p], Tb1 = a.Tb1[p];
    double epsb[3], devb[3];
    double cb = 0.0, depsb = epsb1, qb = 0.0, trb = 0.0;
    for (int k = 0; k < 3; ++k) {
      epsb[k] = Bt[k] * 2.0 * (bm1[k] + 1.0);
      trb += M.K * Tt[k];
      devb[k] = 2.0 * M.mu * (1.0 - c) * Tt[k] - c * epsb[k];
      cb += -2.0 * M.mu * dev[k] * Tt[k] - dev[k] * epsb[k];
    }
    double ebnb = epsb1, Tnb = Tb1;
    if (M.model == OTM_J2_JC) {
      // T' = T_n + chi (1 - c) q deps / (rho0 Cp)
      cb += -M.chi * q * deps / M.rhoCp * Tb1;
      depsb += M.chi * (1.0 - c) * q / M.rhoCp * Tb1;
      qb += M.chi * (1.0 - c) * deps / M.rhoCp * Tb1;
    }
    for (int k = 0; k < kTheta; ++k) thb[k] = 0.0;
    if (plastic) {
      // c = 3 mu deps / q
      depsb += cb * 3.0 * M.mu / q;
      qb -= cb * c / q;
      // deps(q, epsbar_n, T*, theta) from q - 3 mu x - sigma_Y(ebn + x, x/dt, T*) = 0
      qb += depsb * (-1.0 / gx);
      ebnb += depsb * P.s_eb / gx;
      if (M.model == OTM_J2_JC && tunc > 0.0 && tunc < 1.0)
        Tnb += depsb * P.s_T / gx / (M.Tm - M.Tr);
      for (int k = 0; k < kTheta; ++k) thb[k] = depsb * P.s_th[k] / gx;
    }
    a.epsb[p] = ebnb;
    a.Tb[p] = Tnb;
    // q = 2 mu sqrt(3/2 sum dev^2)
    if (q > 0.0)
      for (int k = 0; k < 3; ++k) devb[k] += qb * 6.0 * M.mu * M.mu * dev[k] / q;
    const double devb_sum = devb[0] + devb[1] + devb[2];
    // full adjoint of b_tr - 1 in the eigen-basis: diagonal from the scalar
    // chain, off-diagonal from divided differences of tau_a and bm1_a
    for (int k = 0; k < 3; ++k) {
      const double eb = epsb[k] + trb + devb[k] - devb_sum / 3.0;
      Dt[k] = eb * 0.5 / (1.0 + d[k]);
    }
    for (int k = 3; k < 6; ++k) Dt[k] = Tt[k] * rt[k - 3] + Bt[k] * rbm[k - 3];
  }
  // back to the lab frame: Db = V Dt V^T
  double Db[3][3];
  {
    double Df[3][3];
    for (int k = 0; k < 6; ++k) Df[kVi[k]][kVj[k]] = Df[kVj[k]][kVi[k]] = Dt[k];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int aa = 0; aa < 3; ++aa)
          for (int bb = 0; bb < 3; ++bb) s += V[i][aa] * Df[aa][bb] * V[j][bb];
        Db[i][j] = s;
      }
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage 4: b_tr = dF b^e_n dF^T
  {
    double be[3][3];
    {
      double bd[6];
      for (int k = 0; k < 6; ++k) bd[k] = a.bed[k * n + p];
      for (int k = 0; k < 6; ++k)
        be[kVi[k]][kVj[k]] = be[kVj[k]][kVi[k]] = bd[k] + (k < 3 ? 1.0 : 0.0);
    }
    double DbF[3][3], DbFbe[3][3];
    mat3_mul(Db, dF, DbF);
    mat3_mul(DbF, be, DbFbe);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) dFb[i][j] = 2.0 * DbFbe[i][j];
  }
  {
    double FtDb[3][3], BeB[3][3], bedb[6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) FtDb[i][j] = dF[0][i] * Db[0][j] + dF[1][i] * Db[1][j] + dF[2][i] * Db[2][j];
    mat3_mul(FtDb, dF, BeB);
    full_bar_to_voigt(BeB, bedb);
    for (int k = 0; k < 6; ++k) a.bedb[k * n + p] = bedb[k];
  }
  __builtin_amdgcn_sched_barrier(0);

  // ---- stage 5: J' = det F', F' = dF F_n
  {
    double Fn[3][3], Fp[3][3], cofp[3][3], Fpb[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Fn[i][j] = a.Fd[(3 * i + j) * n + p] + (i == j ? 1.0 : 0.0);
    mat3_mul(dF, Fn, Fp);
    cofactor3(Fp, cofp);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Fpb[i][j] = a.Fdb1[(3 * i + j) * n + p] + Jpb * cofp[i][j];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        dFb[i][j] += Fpb[i][0] * Fn[j][0] + Fpb[i][1] * Fn[j][1] + Fpb[i][2] * Fn[j][2];
        a.Fdb[(3 * i + j) * n + p] = dF[0][i] * Fpb[0][j] + dF[1][i] * Fpb[1][j] + dF[2][i] * Fpb[2][j];
      }
  }
}

__global__ __launch_bounds__(kAdjMpBlock) void k_adj_mp(AdjMpArgs a) {
  __shared__ double sums[9][kAdjMpBlock];   // dF - 1 of the workgroup's MPs
  __shared__ double thred[kTheta][kAdjMpBlock];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)xcd_block() * kAdjMpBlock;
  const int lane = tid % kAdjGather;
  constexpr int groups = kAdjMpBlock / kAdjGather;
  // phase 1: H = dF - 1 = sum du'_I (x) grad N_I
  for (int r = 0; r < kAdjMpBlock / groups; ++r) {
    const int local = r * groups + tid / kAdjGather;
    const int64_t p = base + local;
    double h[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (p < a.n_mp) {
      // kAdjGatherSlots pairs per lane at a time, all loads issued before the
      // first use (slots past the support reload pair q0 and are not used)
      constexpr int L = kAdjGather, S = kAdjGatherSlots;
      const int64_t q0 = a.off[p], q1 = a.off[p + 1];
      const double* recd = reinterpret_cast<const double*>(a.nrec);
      for (int64_t base = q0; base < q1; base += L * S) {
        int32_t I[S];
        double g[S][3], u[S][3];
#pragma unroll
        for (int k = 0; k < S; ++k) {
          const int64_t q = base + k * L + lane;
          const int64_t qq = q < q1 ? q : q0;
          I[k] = a.idx[qq];
          g[k][0] = a.dN[qq];
          g[k][1] = a.dN[a.stride + qq];
          g[k][2] = a.dN[2 * a.stride + qq];
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
          u[k][0] = recd[8 * (int64_t)I[k] + 3];
          const double2 r1 = reinterpret_cast<const double2*>(a.nrec)[4 * (int64_t)I[k] + 2];
          u[k][1] = r1.x;
          u[k][2] = r1.y;
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
          if (base + k * L + lane >= q1) continue;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) h[3 * i + j] += u[k][i] * g[k][j];
        }
      }
    }
    for (int c = 0; c < 9; ++c) h[c] = group_sum<kAdjGather>(h[c]);
    if (lane == 0)
      for (int c = 0; c < 9; ++c) sums[c][local] = h[c];
  }
  __syncthreads();
  // phase 2: one lane per MP
  double th[kTheta] = {0, 0, 0, 0, 0};
  {
    const int64_t p = base + tid;
    if (p < a.n_mp) {
      double dF[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dF[i][j] = sums[3 * i + j][tid] + (i == j ? 1.0 : 0.0);
      double dFb[3][3];
      bool ok;
      mp_adjoint(a, p, dF, dFb, th, ok);
      if (!ok) diag_fail(a.diag, OTM_ERR_RM_NOCONV, (uint64_t)p);
      // v' = det(dF) v
      double cof[3][3];
      cofactor3(dF, cof);
      const double detdF = det3m(dF);
      const double vb1 = a.volb1[p];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) dFb[i][j] += vb1 * a.vol[p] * cof[i][j];
      a.volb[p] = vb1 * detdF;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a.dfb[(3 * i + j) * a.n_mp + p] = dFb[i][j];
    }
  }
  for (int k = 0; k < kTheta; ++k) thred[k][tid] = th[k];
  __syncthreads();
  // parameter gradient: one partial per workgroup
  for (int o = kAdjMpBlock / 2; o > 0; o >>= 1) {
    if (tid < o)
      for (int k = 0; k < kTheta; ++k) thred[k][tid] += thred[k][tid + o];
    __syncthreads();
  }
  if (tid == 0)
    for (int k = 0; k < kTheta; ++k) a.theta_part[blockIdx.x * kTheta + k] = thred[k][0];
}

// ------------------------------------------- K3b: MP update, node adjoints
// Per pair of state n: x_p' = sum N_I x_I' gives x_I' the term N_I x_p'_bar and
// dF = 1 + sum du_I' (x) grad N_I gives du_I' the term dF_bar grad N_I, both
// pre-summed per node in LDS (256 consecutive MPs per workgroup share most of
// their nodes) and then added with one float64 atomic per node and value.
constexpr int kAdjScatMPs = 256;
constexpr int kAdjScatLanes = 8;
constexpr int kAdjScatSlots = 4;
constexpr int kAdjScatBits = 10;

struct AdjScatArgs {
  int64_t n_nodes, n_mp, stride;
  const int64_t* off;
  const int32_t* idx;
  const double* N;
  const double* dN;
  const double* xpb1;  // adjoint of x_p' [3][n_mp]
  const double* dfb;   // adjoint of dF [9][n_mp]
  double* xb1;         // node adjoints of state n+1 (accumulated)
  double* dub1;
};

__global__ __launch_bounds__(256) void k_adj_mp_scatter(AdjScatArgs a) {
  __shared__ NodeSums<6, kAdjScatBits> tab;
  sums_clear(tab);
  __syncthreads();
  double* const dst[6] = {a.xb1, a.xb1 + a.n_nodes, a.xb1 + 2 * a.n_nodes,
                          a.dub1, a.dub1 + a.n_nodes, a.dub1 + 2 * a.n_nodes};
  const int64_t base = (int64_t)xcd_block() * kAdjScatMPs;
  const int lane = threadIdx.x % kAdjScatLanes;
  for (int r = 0; r < kAdjScatMPs / (256 / kAdjScatLanes); ++r) {
    const int64_t p = base + r * (256 / kAdjScatLanes) + threadIdx.x / kAdjScatLanes;
    if (p >= a.n_mp) continue;
    const int64_t n = a.n_mp;
    const double xpb[3] = {a.xpb1[p], a.xpb1[n + p], a.xpb1[2 * n + p]};
    double Fb[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Fb[i][j] = a.dfb[(3 * i + j) * n + p];
    for (int c = 0; c < 3; ++c) hold(xpb[c]);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) hold(Fb[i][j]);
    // kAdjScatSlots pairs per lane at a time, loads first (slots past the
    // support reload pair q0 and are not used)
    constexpr int L = kAdjScatLanes, S = kAdjScatSlots;
    const int64_t q0 = a.off[p], q1 = a.off[p + 1];
    for (int64_t base = q0; base < q1; base += L * S) {
      int32_t I[S];
      double w[S], g[S][3];
#pragma unroll
      for (int k = 0; k < S; ++k) {
        const int64_t q = base + k * L + lane;
        const int64_t qq = q < q1 ? q : q0;
        I[k] = a.idx[qq];
        w[k] = a.N[qq];
        g[k][0] = a.dN[qq];
        g[k][1] = a.dN[a.stride + qq];
        g[k][2] = a.dN[2 * a.stride + qq];
      }
      // one wait for the chunk, before the per-slot branches
#pragma unroll
      for (int k = 0; k < S; ++k) {
        hold(I[k]); hold(w[k]);
        hold(g[k][0]); hold(g[k][1]); hold(g[k][2]);
      }
#pragma unroll
      for (int k = 0; k < S; ++k) {
        if (base + k * L + lane >= q1) continue;
        double c[6];
        for (int i = 0; i < 3; ++i) {
          c[i] = w[k] * xpb[i];
          c[3 + i] = Fb[i][0] * g[k][0] + Fb[i][1] * g[k][1] + Fb[i][2] * g[k][2];
        }
        sums_add(tab, I[k], c, dst);
      }
    }
  }
  __syncthreads();
  sums_flush(tab, dst);
}

// ----------------------------------------------------------- K5: nodes
struct AdjNodeArgs {
  int64_t n;
  const double* x;    // state n
  const double* du;
  const double* m;
  const double* f;
  const double* xb1;  // adjoint of x_{n+1}, du_{n+1}
  const double* dub1;
  double* xb;         // out: adjoint of x_n, du_n
  double* dub;
  double4* fmb;       // out: adjoints of f_n and m_n per node (f_x, f_y, f_z, m)
  double dt2;
  int wall;
  double wx[3], wn[3];
};

__global__ __launch_bounds__(256) void k_adj_node(AdjNodeArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  const double mi = a.m[i];
  double fv[3], pred[3], xs[3], xb1[3], dub1[3];
  const bool has_mass = mi > 0.0;
  for (int c = 0; c < 3; ++c) {
    fv[c] = a.f[c * n + i];
    pred[c] = a.du[c * n + i] + (has_mass ? a.dt2 * fv[c] / mi : 0.0);
    xs[c] = a.x[c * n + i] + pred[c];
    xb1[c] = a.xb1[c * n + i];
    dub1[c] = a.dub1[c * n + i];
  }
  double xb[3], pb[3];  // adjoints of x_n and of the predicted increment
  bool hit = false;
  if (a.wall) {
    const double g = (xs[0] - a.wx[0]) * a.wn[0] + (xs[1] - a.wx[1]) * a.wn[1] + (xs[2] - a.wx[2]) * a.wn[2];
    hit = g < 0.0;
  }
  if (!hit) {
    // du' = pred, x' = x + du'
    for (int c = 0; c < 3; ++c) {
      xb[c] = xb1[c];
      pb[c] = dub1[c] + xb1[c];
    }
  } else {
    // x' = P x* + (x_w . n) n with P = 1 - n n^T, x* = x + pred, du' = x' - x
    double t[3];
    for (int c = 0; c < 3; ++c) t[c] = xb1[c] + dub1[c];
    const double tn = t[0] * a.wn[0] + t[1] * a.wn[1] + t[2] * a.wn[2];
    double xsb[3];
    for (int c = 0; c < 3; ++c) xsb[c] = t[c] - tn * a.wn[c];
    for (int c = 0; c < 3; ++c) {
      xb[c] = xsb[c] - dub1[c];
      pb[c] = xsb[c];
    }
  }
  double fm = 0.0, fb[3];
  for (int c = 0; c < 3; ++c) {
    a.xb[c * n + i] = xb[c];
    a.dub[c * n + i] = pb[c];
    fb[c] = has_mass ? a.dt2 / mi * pb[c] : 0.0;
    fm += fv[c] * pb[c];
  }
  a.fmb[i] = make_double4(fb[0], fb[1], fb[2], has_mass ? -a.dt2 * fm / (mi * mi) : 0.0);
}

// ------------------------------------------------------- K6: assembly
struct AdjAsmArgs {
  int64_t n_nodes, n_mp, stride;
  const int64_t* off;
  const int32_t* idx;
  const double* dN;
  const double* vol;
  const double* mass;
  const double* sigma;
  const double4* fmb;   // adjoints of f and m per node (K5)
  const double4* nrec;  // node records of state n+1 (x, y, z, du_x), (du_y, du_z, 0, 0)
  const double* xpb1;  // adjoint of x_p' [3][n_mp]
  const double* dfb;   // adjoint of dF [9][n_mp]
  double* Nb;      // written per pair
  double* dNb;     // written per pair [3][stride]
  double* sigb;    // written
  double* volb;    // +=
};

// Pair adjoints of state n in one pass: N_I enters x_p' = sum N_I x_I' and the
// lumped mass m_I = sum N_I m_p; grad N_I enters dF = 1 + sum du_I' (x) grad N_I
// and the force f_I = -sum v sigma grad N_I.  The MP sums of the force terms
// give the adjoints of sigma and v.
constexpr int kAdjAsmLanes = 8;
constexpr int kAdjAsmSlots = 4;   // pairs per lane whose loads are issued together
__global__ __launch_bounds__(256) void k_adj_assembly(AdjAsmArgs a) {
  constexpr int L = kAdjAsmLanes, S = kAdjAsmSlots;
  const int64_t p = (int64_t)xcd_block() * (256 / L) + threadIdx.x / L;
  const int lane = threadIdx.x % L;
  if (p >= a.n_mp) return;
  const int64_t n = a.n_mp;
  const double v = a.vol[p], mp = a.mass[p];
  double s[6];
  for (int c = 0; c < 6; ++c) s[c] = a.sigma[c * n + p];
  const double xpb[3] = {a.xpb1[p], a.xpb1[n + p], a.xpb1[2 * n + p]};
  double Fb[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Fb[i][j] = a.dfb[(3 * i + j) * n + p];
  hold(v); hold(mp);
  for (int c = 0; c < 6; ++c) hold(s[c]);
  for (int c = 0; c < 3; ++c) hold(xpb[c]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) hold(Fb[i][j]);
  double sb[6] = {0, 0, 0, 0, 0, 0}, vb = 0.0;
  const int64_t q0 = a.off[p], q1 = a.off[p + 1];
  const double2* rec2 = reinterpret_cast<const double2*>(a.nrec);
  // S pairs per lane at a time: every load of the chunk is issued before the
  // first use (slots past the support reload pair q0 and are not used)
  for (int64_t base = q0; base < q1; base += L * S) {
    int32_t I[S];
    double g[S][3];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const int64_t q = base + k * L + lane;
      const int64_t qq = q < q1 ? q : q0;
      I[k] = a.idx[qq];
      g[k][0] = a.dN[qq];
      g[k][1] = a.dN[a.stride + qq];
      g[k][2] = a.dN[2 * a.stride + qq];
    }
    double4 r0[S], fm[S];
    double2 r1[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
      r0[k] = a.nrec[2 * (int64_t)I[k]];
      r1[k] = rec2[4 * (int64_t)I[k] + 2];   // (du_y, du_z)
      fm[k] = a.fmb[I[k]];
    }
    // one wait for the chunk, before the per-slot branches
#pragma unroll
    for (int k = 0; k < S; ++k) {
      hold(r0[k]); hold(r1[k]); hold(fm[k]);
      hold(g[k][0]); hold(g[k][1]); hold(g[k][2]);
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
      const int64_t q = base + k * L + lane;
      if (q >= q1) continue;
      const double f[3] = {fm[k].x, fm[k].y, fm[k].z};
      const double u[3] = {r0[k].w, r1[k].x, r1[k].y};
      a.Nb[q] = r0[k].x * xpb[0] + r0[k].y * xpb[1] + r0[k].z * xpb[2] + fm[k].w * mp;
      // f_I = -v sigma g
      const double sf[3] = {s[0] * f[0] + s[3] * f[1] + s[5] * f[2],
                            s[3] * f[0] + s[1] * f[1] + s[4] * f[2],
                            s[5] * f[0] + s[4] * f[1] + s[2] * f[2]};
      for (int j = 0; j < 3; ++j)
        a.dNb[j * a.stride + q] = Fb[0][j] * u[0] + Fb[1][j] * u[1] + Fb[2][j] * u[2] - v * sf[j];
      vb -= sf[0] * g[k][0] + sf[1] * g[k][1] + sf[2] * g[k][2];
      sb[0] -= v * f[0] * g[k][0];
      sb[1] -= v * f[1] * g[k][1];
      sb[2] -= v * f[2] * g[k][2];
      sb[3] -= v * (f[0] * g[k][1] + f[1] * g[k][0]);
      sb[4] -= v * (f[1] * g[k][2] + f[2] * g[k][1]);
      sb[5] -= v * (f[0] * g[k][2] + f[2] * g[k][0]);
    }
  }
  for (int c = 0; c < 6; ++c) sb[c] = group_sum<L>(sb[c]);
  vb = group_sum<L>(vb);
  if (lane == 0) {
    for (int c = 0; c < 6; ++c) a.sigb[c * n + p] = sb[c];
    a.volb[p] += vb;
  }
}

__global__ __launch_bounds__(256) void k_adj_theta(const double* part, int64_t nb,
                                                   double* theta_bar) {
  __shared__ double red[kTheta][256];
  double s[kTheta] = {0, 0, 0, 0, 0};
  for (int64_t b = threadIdx.x; b < nb; b += 256)
    for (int k = 0; k < kTheta; ++k) s[k] += part[b * kTheta + k];
  for (int k = 0; k < kTheta; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int k = 0; k < kTheta; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < kTheta; ++k) theta_bar[k] += red[k][0];
}

// ------------------------------------------ start of the central difference
// du_0 = dt v0: v0_bar = dt du_bar per node and component.
__global__ __launch_bounds__(256) void k_v0_bar(int64_t n3, double dt,
                                                const double* __restrict__ dub,
                                                double* __restrict__ v0b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n3) v0b[i] = dt * dub[i];
}

// sum_i v0b_i dir_i by one workgroup: each thread sums a fixed strided set,
// then a fixed tree, so the result does not depend on scheduling.
__global__ __launch_bounds__(1024) void k_dir_dot(int64_t n3, const double* __restrict__ v0b,
                                                  const double* __restrict__ dir,
                                                  double* __restrict__ out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n3; i += 1024) acc += v0b[i] * dir[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

void launch_init_adjoint(int64_t n_nodes, double dt, const double* du_bar, double* v0_bar,
                         const double* dir, double* dir_bar, hipStream_t s) {
  const int64_t n3 = 3 * n_nodes;
  if (n3 > 0) k_v0_bar<<<(unsigned)((n3 + 255) / 256), 256, 0, s>>>(n3, dt, du_bar, v0_bar);
  if (dir_bar != nullptr) k_dir_dot<<<1, 1024, 0, s>>>(n3, v0_bar, dir, dir_bar);
}

// ------------------------------------------------------------ host side
size_t adjoint_workspace_bytes(int64_t n_nodes, int64_t n_mp) {
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const int64_t nb = (n_mp + kAdjMpBlock - 1) / kAdjMpBlock + 1;
  return al(sizeof(double) * 3 * (size_t)n_mp) + al(sizeof(double4) * (size_t)n_nodes) +
         al(sizeof(double) * kTheta * (size_t)nb) + al(sizeof(double) * 9 * (size_t)n_mp) +
         al(sizeof(double4) * 2 * (size_t)n_nodes);
}

void launch_step_adjoint(const otm_tape& t0, const otm_tape& t1, const otm_params& p,
                         double dt, const double* mass, otm_state_bar& b1, otm_state_bar& b0,
                         double* theta_bar, void* ws, otm_diag* diag, hipStream_t s) {
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const int64_t nn = t0.n_nodes, nm = t0.n_mp;
  char* c = (char*)ws;
  double* xpb = (double*)c;
  c += al(sizeof(double) * 3 * (size_t)nm);
  double4* fmb = (double4*)c;
  c += al(sizeof(double4) * (size_t)nn);
  double* theta_part = (double*)c;
  c += al(sizeof(double) * kTheta * (size_t)((nm + kAdjMpBlock - 1) / kAdjMpBlock + 1));
  double* dfb = (double*)c;
  c += al(sizeof(double) * 9 * (size_t)nm);
  double4* nrec = (double4*)c;

  if (nm > 0 && nn > 0) {
    // node records of state n+1, the forward's layout
    otm_state ns{};
    ns.n_nodes = nn;
    ns.x = const_cast<double*>(t1.x);
    ns.du = const_cast<double*>(t1.du);
    launch_pack_nodes(ns, nrec, s);
  }
  if (nm > 0) {
    // K1: shape functions of state n+1
    AdjLmeArgs la{nn, nm, t1.pair_stride, nrec, t1.xp, t1.lam, t1.nbr_offsets, t1.nbr_idx,
                  b1.N, b1.dN, p.beta, xpb, b1.x, diag};
    const int per = (256 / kAdjG) * kAdjLmeRounds;
    k_adj_lme<kAdjG, kAdjPPL, 0, false><<<(unsigned)((nm + per - 1) / per), 256, 0, s>>>(la);
    const int per_long = (256 / kAdjLongG) * kAdjLmeRounds;
    k_adj_lme<kAdjLongG, kAdjLongPPL, kAdjG * kAdjPPL, true>
        <<<(unsigned)((nm + per_long - 1) / per_long), 256, 0, s>>>(la);
    // K3: MP update per MP (adjoint of dF to the workspace), then its node terms
    AdjMpArgs ma;
    ma.n_nodes = nn; ma.n_mp = nm; ma.stride = t0.pair_stride;
    ma.off = t0.nbr_offsets; ma.idx = t0.nbr_idx; ma.N = t0.N; ma.dN = t0.dN;
    ma.vol = t0.vol; ma.Fd = t0.Fd; ma.bed = t0.bed; ma.epsbar = t0.epsbar; ma.T = t0.T;
    ma.nrec = nrec;
    ma.xpb1 = xpb; ma.volb1 = b1.vol; ma.Fdb1 = b1.Fd; ma.bedb1 = b1.bed; ma.epsb1 = b1.epsbar;
    ma.Tb1 = b1.T; ma.sigb1 = b1.sigma;
    ma.volb = b0.vol; ma.Fdb = b0.Fd; ma.bedb = b0.bed; ma.epsb = b0.epsbar; ma.Tb = b0.T;
    ma.dfb = dfb;
    ma.theta_part = theta_part;
    ma.M = make_mat<double>(p, dt);
    ma.dt = dt;
    ma.diag = diag;
    const unsigned nbm = (unsigned)((nm + kAdjMpBlock - 1) / kAdjMpBlock);
    k_adj_mp<<<nbm, kAdjMpBlock, 0, s>>>(ma);
    k_adj_theta<<<1, 256, 0, s>>>(theta_part, nbm, theta_bar);
    AdjScatArgs sa{nn, nm, t0.pair_stride, t0.nbr_offsets, t0.nbr_idx, t0.N, t0.dN,
                   xpb, dfb, b1.x, b1.du};
    k_adj_mp_scatter<<<(unsigned)((nm + kAdjScatMPs - 1) / kAdjScatMPs), 256, 0, s>>>(sa);
  }
  if (nn > 0) {
    // K5: node update
    AdjNodeArgs na;
    na.n = nn; na.x = t0.x; na.du = t0.du; na.m = t0.m; na.f = t0.f;
    na.xb1 = b1.x; na.dub1 = b1.du; na.xb = b0.x; na.dub = b0.du; na.fmb = fmb;
    na.dt2 = dt * dt;
    na.wall = p.wall_enabled;
    for (int k = 0; k < 3; ++k) { na.wx[k] = p.wall_x[k]; na.wn[k] = p.wall_n[k]; }
    k_adj_node<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(na);
  }
  if (nm > 0) {
    // K6: pair adjoints of state n, and the adjoints of sigma and v
    AdjAsmArgs aa{nn, nm, t0.pair_stride, t0.nbr_offsets, t0.nbr_idx, t0.dN, t0.vol,
                  mass, t0.sigma, fmb, nrec, xpb, dfb, b0.N, b0.dN, b0.sigma, b0.vol};
    k_adj_assembly<<<(unsigned)((nm + (256 / kAdjAsmLanes) - 1) / (256 / kAdjAsmLanes)), 256, 0,
                     s>>>(aa);
  }
}

}  // namespace otm
