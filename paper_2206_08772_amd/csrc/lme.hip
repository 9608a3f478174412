// Local max-ent shape functions (Sec. 2.3) by a per-material-point damped
// Newton solve for the Lagrange multiplier, in float64.
//
// A group of G = 4 lanes works on one MP; each lane keeps up to PPL = 9 of
// the MP's pairs in registers (offset d = x_p - x_I), so one Newton
// evaluation costs one exp per pair and 10 group reductions (Z, r,
// S = sum e d d^T) of two DPP stages each.  The 3x3 solve is repeated in
// every lane of the group, so the group never diverges.  Few lanes per MP
// keep the per-MP work (reductions, solve, line search) from being repeated
// across many lanes; the kernel is bound by the latency of that per-MP chain
// at two waves per SIMD, not by memory traffic.  The supports of the
// lattice-like bodies hold 20-33 nodes (radius 1.86 h), up to 35 where the
// rod is compressed; MPs with more than 36 pairs take the same iteration
// with pairs re-read from memory, which is several times slower, and since
// such MPs cluster in space the workgroup holding them sets the kernel's
// end (with 32 cached pairs the rod's 0.03 % of MPs with 33-35 pairs cost
// 13 % of the kernel after 100 steps).
//
// Newton reading (the paper gives none): start from the previous multiplier;
// step -J^{-1} r with J = sum N d d^T - r r^T; Armijo backtracking on log Z
// with sufficient-decrease factor 1e-4 plus a round-off allowance
// 1e-12 (1 + |log Z|), up to 30 halvings; stop at |r|_2 <= tol.  Gradients
// dN_I = -N_I J^{-1} d_I at the converged multiplier.
#include "launch.h"
#include "otm_common.h"

namespace otm {

// Node coordinates: SoA arrays, or the packed (x, y, z, 0) records the step
// keeps in its workspace (one 32-byte load per node).
struct NodeSrc {
  const double* x;       // [3][n] (used when packed == nullptr)
  const double4* packed; // record 2 I = (x, y, z, du_x)
  int64_t n;
};
OTM_DEV void node_xyz(const NodeSrc& s, int32_t I, double& a, double& b, double& c) {
  if (s.packed != nullptr) {
    const double4 v = s.packed[2 * (int64_t)I];
    a = v.x; b = v.y; c = v.z;
  } else {
    a = s.x[I]; b = s.x[s.n + I]; c = s.x[2 * s.n + I];
  }
}

// exp(x) for the shifted exponents of the LME weights (x <= 0 up to
// rounding): Cody-Waite reduction x = k ln2 + r with ln2 split in a 32-bit
// head and its remainder (k ln2_hi is exact), |r| <= ln2/2, then the Taylor
// polynomial of degree 12 in Horner form (truncation below 2e-16 relative on
// that range) and a scale by 2^k; 0 below -745.  The coefficients sit in
// constant memory, so they reach the FMAs from scalar registers.
__constant__ double kExpTaylor[13] = {
    1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664, 0.008333333333333333,
    0.001388888888888889, 0.0001984126984126984, 2.48015873015873e-05,
    2.7557319223985893e-06, 2.755731922398589e-07, 2.505210838544172e-08,
    2.08767569878681e-09};
OTM_DEV double lme_exp(double x) {
  const double k = rint(x * 1.4426950408889634);
  double r = fma(k, -0.6931471803691238, x);
  r = fma(k, -1.9082149292705877e-10, r);
  double p = kExpTaylor[12];
#pragma unroll
  for (int i = 11; i >= 0; --i) p = fma(p, r, kExpTaylor[i]);
  const double e = ldexp(p, (int)k);
  return x < -745.0 ? 0.0 : e;
}

struct Eval {
  double logZ, Z, fmax;
  double r[3];
  double J[6];  // xx yy zz xy yz xz
};

template <int G, int PPL, bool CACHED>
struct Pairs {
  // cached offsets x_p - x_I (CACHED only); the prior -beta |d|^2 is
  // recomputed from them at each evaluation, which costs fewer cycles than
  // the registers it would hold
  double d[CACHED ? PPL : 1][3];
};

// A row of the support lists fetched ahead of its solve: its start and
// the next row's start, its length (taken from the two only once the ids are
// fetched, so that no wait follows the offsets' load) and, for rows of at
// most G * PPL pairs, this lane's node ids.
template <int PPL>
struct RowIds {
  int64_t off, end;
  int K;
  int32_t I[PPL];
};

template <int G, int PPL, bool CACHED>
OTM_DEV void lme_eval(const Pairs<G, PPL, CACHED>& pr, int lane, int K, int64_t off,
                      const double px, const double py, const double pz, const NodeSrc& ns,
                      const int32_t* __restrict__ idx, double beta, const double lam[3],
                      Eval& ev, double ek[CACHED ? PPL : 1]) {
  double fm = -INFINITY;
  if constexpr (CACHED) {
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      if (k * G + lane < K) {
        const double prior = -beta * ((pr.d[k][0] * pr.d[k][0] + pr.d[k][1] * pr.d[k][1]) +
                                      pr.d[k][2] * pr.d[k][2]);
        ek[k] = prior + (lam[0] * pr.d[k][0] + lam[1] * pr.d[k][1] + lam[2] * pr.d[k][2]);
        fm = fmax(fm, ek[k]);
      }
    }
  } else {
    for (int q = lane; q < K; q += G) {
      const int32_t I = idx[off + q];
      double nx, ny, nz;
      node_xyz(ns, I, nx, ny, nz);
      const double dx = px - nx, dy = py - ny, dz = pz - nz;
      const double f = -beta * ((dx * dx + dy * dy) + dz * dz) + (lam[0] * dx + lam[1] * dy + lam[2] * dz);
      fm = fmax(fm, f);
    }
  }
  fm = group_max<G>(fm);
  double Z = 0, r0 = 0, r1 = 0, r2 = 0, s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0, s5 = 0;
  auto accum = [&](double e, double dx, double dy, double dz) {
    Z += e;
    r0 += e * dx; r1 += e * dy; r2 += e * dz;
    s0 += e * dx * dx; s1 += e * dy * dy; s2 += e * dz * dz;
    s3 += e * dx * dy; s4 += e * dy * dz; s5 += e * dx * dz;
  };
  if constexpr (CACHED) {
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      if (k * G + lane < K) {
        ek[k] = lme_exp(ek[k] - fm);
        accum(ek[k], pr.d[k][0], pr.d[k][1], pr.d[k][2]);
      }
    }
  } else {
    for (int q = lane; q < K; q += G) {
      const int32_t I = idx[off + q];
      double nx, ny, nz;
      node_xyz(ns, I, nx, ny, nz);
      const double dx = px - nx, dy = py - ny, dz = pz - nz;
      const double f = -beta * ((dx * dx + dy * dy) + dz * dz) + (lam[0] * dx + lam[1] * dy + lam[2] * dz);
      accum(lme_exp(f - fm), dx, dy, dz);
    }
  }
  Z = group_sum<G>(Z);
  r0 = group_sum<G>(r0); r1 = group_sum<G>(r1); r2 = group_sum<G>(r2);
  s0 = group_sum<G>(s0); s1 = group_sum<G>(s1); s2 = group_sum<G>(s2);
  s3 = group_sum<G>(s3); s4 = group_sum<G>(s4); s5 = group_sum<G>(s5);
  const double iz = 1.0 / Z;
  ev.Z = Z;
  ev.fmax = fm;
  ev.logZ = log(Z) + fm;
  ev.r[0] = r0 * iz; ev.r[1] = r1 * iz; ev.r[2] = r2 * iz;
  ev.J[0] = s0 * iz - ev.r[0] * ev.r[0];
  ev.J[1] = s1 * iz - ev.r[1] * ev.r[1];
  ev.J[2] = s2 * iz - ev.r[2] * ev.r[2];
  ev.J[3] = s3 * iz - ev.r[0] * ev.r[1];
  ev.J[4] = s4 * iz - ev.r[1] * ev.r[2];
  ev.J[5] = s5 * iz - ev.r[0] * ev.r[2];
}

template <typename DN>
OTM_DEV void store_dn(DN* dN, int64_t cap, int64_t q, const double g[3]) {
  dN[q] = (DN)g[0];
  dN[cap + q] = (DN)g[1];
  dN[2 * cap + q] = (DN)g[2];
}

// What happens to each finished pair besides storing N and grad N.
struct NoSink {
  static constexpr bool kBatch = false;
  OTM_DEV void begin(int64_t) {}
  OTM_DEV void ready() const {}
  OTM_DEV void operator()(int64_t, double, const double*) {}
};

// Fused nodal assembly (nodal mass and residual equations, Sec. 2.1): the
// pair's m and f contributions, with the same arithmetic as the standalone
// assembly kernel (grad N rounded to its stored type R first), go into the
// workgroup's node table.  With conduction (HEAT) the table also sums
// N m_p T_p and v_p q_p . grad N (float64, grad N rounded the same way).
// begin() loads the MP's mass, volume, stress (and temperature and flux)
// once the Newton solve is done.
template <typename R, bool HEAT, typename Q>
struct AsmSink {
  static constexpr bool kBatch = true;  // the cached path inserts a batch of pairs at once
  static constexpr int V = HEAT ? 6 : 4;
  NodeTableV<V>* t;
  const int32_t* idx;
  const double* vol;
  const double* mass;
  const R* sigma;
  const double* Tmp;
  const double* q;
  NodeDst<V> dst;
  int64_t n_mp;
  double mp, vd, Tp, q0, q1, q2;
  R s0, s1, s2, s3, s4, s5;
  OTM_DEV void begin(int64_t p) {
    mp = mass[p];
    vd = vol[p];
    s0 = sigma[p]; s1 = sigma[n_mp + p]; s2 = sigma[2 * n_mp + p];
    s3 = sigma[3 * n_mp + p]; s4 = sigma[4 * n_mp + p]; s5 = sigma[5 * n_mp + p];
    if constexpr (HEAT) {
      Tp = Tmp[p];
      q0 = q[p]; q1 = q[n_mp + p]; q2 = q[2 * n_mp + p];
    }
  }
  // The values loaded by begin() are first used inside the per-pair
  // branches, where the compiler waits for them with a full wait that also
  // waits for every store issued so far (N, grad N of the earlier pairs);
  // holding them here puts that one wait in straight-line code before the
  // pairs, so the pairs' stores stay in flight.
  OTM_DEV void ready() const {
    hold(mp); hold(vd);
    hold(s0); hold(s1); hold(s2); hold(s3); hold(s4); hold(s5);
    if constexpr (HEAT) { hold(Tp); hold(q0); hold(q1); hold(q2); }
  }
  OTM_DEV void values(double Nq, const double g[3], double (&c)[V]) const {
    const R g0 = (R)g[0], g1 = (R)g[1], g2 = (R)g[2];
    c[0] = Nq * mp;
    pair_force<Q>(vd, s0, s1, s2, s3, s4, s5, g0, g1, g2, c[1], c[2], c[3]);
    if constexpr (HEAT) {
      c[4] = c[0] * Tp;
      c[5] = vd * ((q0 * (double)g0 + q1 * (double)g1) + q2 * (double)g2);
    }
  }
  OTM_DEV void operator()(int64_t q_, double Nq, const double g[3]) {
    double c[V];
    values(Nq, g, c);
    table_insert<V>(*t, idx[q_], c, dst);
  }
  template <int NB>
  OTM_DEV void insert(const int32_t (&I)[NB], const bool (&use)[NB], const double (&c)[NB][V]) {
    table_insert_batch<V, NB>(*t, I, use, c, dst);
  }
};

// Fused contribution store of the deterministic assembly: the pair's four
// contributions (the standalone contribution kernel's arithmetic) go to its
// place in the node-sorted order, where each node later sums them in order.
template <typename R, typename Q>
struct SegSink {
  static constexpr bool kBatch = false;
  const double* vol;
  const double* mass;
  const R* sigma;
  const int32_t* pos_of;
  double4* contrib;
  int64_t n_mp;
  double mp, vd;
  R s0, s1, s2, s3, s4, s5;
  OTM_DEV void begin(int64_t p) {
    mp = mass[p];
    vd = vol[p];
    s0 = sigma[p]; s1 = sigma[n_mp + p]; s2 = sigma[2 * n_mp + p];
    s3 = sigma[3 * n_mp + p]; s4 = sigma[4 * n_mp + p]; s5 = sigma[5 * n_mp + p];
  }
  // as AsmSink::ready
  OTM_DEV void ready() const {
    hold(mp); hold(vd);
    hold(s0); hold(s1); hold(s2); hold(s3); hold(s4); hold(s5);
  }
  OTM_DEV void operator()(int64_t q, double Nq, const double g[3]) {
    const R g0 = (R)g[0], g1 = (R)g[1], g2 = (R)g[2];
    double c1, c2, c3;
    pair_force<Q>(vd, s0, s1, s2, s3, s4, s5, g0, g1, g2, c1, c2, c3);
    contrib[pos_of[q]] = make_double4(Nq * mp, c1, c2, c3);
  }
};

// Fetch this lane's node ids of a row whose bounds are set (rows longer than
// G * PPL take the uncached path, which reads its ids itself).
template <int G, int PPL>
OTM_DEV void load_row_ids(RowIds<PPL>& r, const int32_t* __restrict__ idx, int lane) {
  r.K = (int)(r.end - r.off);
  if (r.K > 0 && r.K <= G * PPL) {
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int q = k * G + lane;
      r.I[k] = idx[r.off + (q < r.K ? q : 0)];
    }
  }
}

// Waits for a fetched row in straight-line code.  A row still in flight
// where control paths join (the end of a round) gets a full wait there, which
// also waits for every store of the round.  (Its bounds were waited for when
// its length was taken.)
template <int PPL>
OTM_DEV void hold_row(const RowIds<PPL>& r) {
  hold(r.K);
#pragma unroll
  for (int k = 0; k < PPL; ++k) hold(r.I[k]);
}

struct NoMid {
  OTM_DEV void operator()() const {}
  OTM_DEV void ready() const {}
};

// Two hooks into an MP's solve: ``fetch`` once the Newton iteration has
// ended, ``wait`` where the MP's own assembly loads are waited for.
template <class F, class W>
struct MidHooks {
  F fetch;
  W wait;
  OTM_DEV void operator()() const { fetch(); }
  OTM_DEV void ready() const { wait(); }
};

// One MP's solve.  ``pre`` (nullable) holds the row fetched ahead; ``mid``
// runs once the Newton iteration has ended (the fused kernel fetches the
// next round's node ids there, so they arrive while this MP finishes) and
// ``mid.ready()`` where the MP's own assembly loads are waited for.
template <int G, int PPL, bool CACHED, typename DN, class Sink, class Mid = NoMid>
OTM_DEV void lme_point(int64_t p, int lane, const NodeSrc& ns, int64_t n_mp, const double* __restrict__ xp,
                       const int64_t* __restrict__ offsets, const int32_t* __restrict__ idx,
                       int64_t cap, double beta, double tol, int max_iter,
                       double* __restrict__ lam_io, double* __restrict__ Nout,
                       DN* __restrict__ dN, otm_diag* diag, Sink& sink,
                       const RowIds<PPL>* pre = nullptr, Mid mid = Mid{}) {
  const int64_t off = pre != nullptr ? pre->off : offsets[p];
  const int K = pre != nullptr ? pre->K : (int)(offsets[p + 1] - off);
  const double px = xp[p], py = xp[n_mp + p], pz = xp[2 * n_mp + p];
  double lam[3] = {lam_io[p], lam_io[n_mp + p], lam_io[2 * n_mp + p]};
  Pairs<G, PPL, CACHED> pr;
  if constexpr (CACHED) {
    // branch-free loads (the MP's first pair stands in for empty slots) so
    // that all of them are in flight together
    if (K > 0) {
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const int q = k * G + lane;
        const int32_t I = pre != nullptr ? pre->I[k] : idx[off + (q < K ? q : 0)];
        double nx, ny, nz;
        node_xyz(ns, I, nx, ny, nz);
        pr.d[k][0] = px - nx;
        pr.d[k][1] = py - ny;
        pr.d[k][2] = pz - nz;
      }
    }
  }
  // the multiplier arrives with the node gathers (one wait for both)
  hold(lam[0]); hold(lam[1]); hold(lam[2]);
  // ek holds the exponentials of the last evaluation; every line search
  // ends with an accepted trial, so they always belong to the current lambda
  double ek[CACHED ? PPL : 1];
  Eval ev;
  lme_eval<G, PPL, CACHED>(pr, lane, K, off, px, py, pz, ns, idx, beta, lam, ev, ek);
  bool converged = false;
  for (int it = 0;; ++it) {
    const double rn = sqrt(ev.r[0] * ev.r[0] + ev.r[1] * ev.r[1] + ev.r[2] * ev.r[2]);
    if (rn <= tol) { converged = true; break; }
    if (it >= max_iter) break;
    double Mi[6], det;
    sym_inv(ev.J, Mi, det);
    const double tr = ev.J[0] + ev.J[1] + ev.J[2];
    if (!(det > 1e-30 * tr * tr * tr) || !isfinite(det)) break;  // multiplier ran away
    double delta[3];
    sym_mul_vec(Mi, ev.r, delta);
    delta[0] = -delta[0]; delta[1] = -delta[1]; delta[2] = -delta[2];
    // only log Z and the slope of the base point are needed from here on, so
    // the trials are evaluated into ev (the accepted one stays there)
    const double slope = ev.r[0] * delta[0] + ev.r[1] * delta[1] + ev.r[2] * delta[2];
    const double lz0 = ev.logZ;
    const double l0[3] = {lam[0], lam[1], lam[2]};
    double t = 1.0;
    for (int h = 0; h < 31; ++h) {
      lam[0] = l0[0] + t * delta[0];
      lam[1] = l0[1] + t * delta[1];
      lam[2] = l0[2] + t * delta[2];
      lme_eval<G, PPL, CACHED>(pr, lane, K, off, px, py, pz, ns, idx, beta, lam, ev, ek);
      if (ev.logZ <= lz0 + 1e-4 * t * slope + 1e-12 * (1.0 + fabs(lz0)) || h == 30) break;
      t *= 0.5;
    }
  }
  mid();
  if (lane == 0) {
    lam_io[p] = lam[0]; lam_io[n_mp + p] = lam[1]; lam_io[2 * n_mp + p] = lam[2];
    if (!converged) diag_fail(diag, OTM_ERR_LME_NOCONV, (uint64_t)p);
  }
  double Mi[6], det;
  sym_inv(ev.J, Mi, det);
  const double iz = 1.0 / ev.Z;
  sink.begin(p);
  sink.ready();
  mid.ready();
  auto finish = [&](int q, double e, double dx, double dy, double dz) {
    const double Nq = e * iz;
    const double d3[3] = {dx, dy, dz};
    double g[3];
    sym_mul_vec(Mi, d3, g);
    g[0] *= -Nq; g[1] *= -Nq; g[2] *= -Nq;
    Nout[off + q] = Nq;
    store_dn<DN>(dN, cap, off + q, g);
    sink(off + q, Nq, g);
  };
  if constexpr (CACHED && Sink::kBatch) {
    // the pairs in two batches (a bound on the registers the contributions
    // hold): N and grad N stored, then the batch's contributions inserted
    constexpr int V = Sink::V, NB = (PPL + 1) / 2;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      int32_t I[NB];
      bool use[NB];
      double c[NB][V];
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int k = b * NB + j;
        const int q = k * G + lane;
        use[j] = k < PPL && q < K;
        I[j] = !use[j] ? 0 : (pre != nullptr ? pre->I[k < PPL ? k : 0] : idx[off + q]);
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int k = b * NB + j;
        if (k < PPL && use[j]) {
          const int q = k * G + lane;
          const double Nq = ek[k] * iz;
          const double d3[3] = {pr.d[k][0], pr.d[k][1], pr.d[k][2]};
          double g[3];
          sym_mul_vec(Mi, d3, g);
          g[0] *= -Nq; g[1] *= -Nq; g[2] *= -Nq;
          Nout[off + q] = Nq;
          store_dn<DN>(dN, cap, off + q, g);
          sink.values(Nq, g, c[j]);
        }
      }
      sink.insert(I, use, c);
    }
  } else if constexpr (CACHED) {
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int q = k * G + lane;
      if (q < K) finish(q, ek[k], pr.d[k][0], pr.d[k][1], pr.d[k][2]);
    }
  } else {
    for (int q = lane; q < K; q += G) {
      const int32_t I = idx[off + q];
      double nx, ny, nz;
      node_xyz(ns, I, nx, ny, nz);
      const double dx = px - nx, dy = py - ny, dz = pz - nz;
      const double f = -beta * ((dx * dx + dy * dy) + dz * dz) + (lam[0] * dx + lam[1] * dy + lam[2] * dz);
      finish(q, lme_exp(f - ev.fmax), dx, dy, dz);
    }
  }
}

template <int G, int PPL, typename DN, class Sink>
__global__ __launch_bounds__(256) void k_lme(NodeSrc ns, int64_t n_mp, const double* __restrict__ xp,
                                             const int64_t* __restrict__ offsets,
                                             const int32_t* __restrict__ idx, int64_t cap,
                                             double beta, double tol, int max_iter,
                                             double* __restrict__ lam, double* __restrict__ N,
                                             DN* __restrict__ dN, otm_diag* diag, Sink sink) {
  constexpr int per_block = 256 / G;
  const int64_t p = (int64_t)xcd_block() * per_block + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (p >= n_mp) return;  // whole group leaves together
  if (offsets[n_mp] > cap) return;  // lists were not written (capacity)
  const int K = (int)(offsets[p + 1] - offsets[p]);
  if (K <= G * PPL)
    lme_point<G, PPL, true, DN>(p, lane, ns, n_mp, xp, offsets, idx, cap, beta, tol,
                                max_iter, lam, N, dN, diag, sink);
  else
    lme_point<G, PPL, false, DN>(p, lane, ns, n_mp, xp, offsets, idx, cap, beta, tol,
                                 max_iter, lam, N, dN, diag, sink);
}

// Shape functions with the atomic nodal assembly fused in.  A fixed grid of
// kLmeAsmBlocks workgroups (two per CU at this kernel's register use) each
// take chunks of `chunk` consecutive MPs (spatially compact) in rounds of
// 256 / G (a chunk's last round may be partial); the node table is flushed
// to m and f every kLmeAsmFlushRounds rounds and at the end of each chunk.
// The round count is the same for every lane of a workgroup, so the barriers
// around a flush are reached by all of them.
constexpr int kLmeAsmBlocks = 512;
constexpr int kLmeAsmFlushRounds = 8;
static_assert(kLmeAsmBlocks % 8 == 0, "the workgroups split evenly over the 8 XCDs");

// Chunk size.  With four or more chunks of 512 MPs per workgroup, 512 (the
// chunks are dealt round-robin); otherwise one contiguous range per
// workgroup, every workgroup busy (smaller chunks would add flushes faster
// than they even out the work).
inline int64_t lme_asm_chunk(int64_t n_mp) {
  const int64_t per_wg = (n_mp + kLmeAsmBlocks - 1) / kLmeAsmBlocks;
  return per_wg >= 4 * 512 ? 512 : per_wg;
}

template <int G, int PPL, typename DN, bool HEAT, typename Q>
__global__ __launch_bounds__(256) void k_lme_asm(NodeSrc ns, int64_t n_mp,
                                                 const double* __restrict__ xp,
                                                 const int64_t* __restrict__ offsets,
                                                 const int32_t* __restrict__ idx, int64_t cap,
                                                 double beta, double tol, int max_iter,
                                                 double* __restrict__ lam,
                                                 double* __restrict__ N, DN* __restrict__ dN,
                                                 otm_diag* diag, AsmIn a, int64_t chunk) {
  constexpr int per_round = 256 / G;
  const int64_t rpc = (chunk + per_round - 1) / per_round;  // rounds per chunk
  using Sink = AsmSink<DN, HEAT, Q>;
  __shared__ NodeTableV<Sink::V> table;
  const int tid = threadIdx.x;
  table_clear(table, tid, 256);
  __syncthreads();
  // Each XCD takes a contiguous eighth of the chunks (its workgroups' gathers
  // then share its L2) and deals them round-robin to its workgroups.  With
  // several chunks per workgroup, a workgroup's chunks come from across its
  // XCD's range, so regions of slow MPs (more pairs, more Newton steps) are
  // shared out instead of setting one workgroup's, and the kernel's, end;
  // with one, each workgroup has a contiguous range.
  const int64_t n_chunks = (n_mp + chunk - 1) / chunk;
  const int64_t xcd = blockIdx.x % 8u, wgs = gridDim.x / 8u, j = blockIdx.x / 8u;
  const int64_t c_lo = n_chunks * xcd / 8, c_hi = n_chunks * (xcd + 1) / 8;
  const bool ok = offsets[n_mp] <= cap;  // lists were written (capacity)
  const int lane = tid % G;
  NodeDst<Sink::V> dst;
  dst.d[0] = a.m;
  dst.d[1] = a.f;
  dst.d[2] = a.f + a.n_nodes;
  dst.d[3] = a.f + 2 * a.n_nodes;
  if constexpr (HEAT) {
    dst.d[4] = a.heat;
    dst.d[5] = a.heat + a.n_nodes;
  }
  Sink sink{&table, idx, a.vol, a.mass, (const DN*)a.sigma, a.T, a.q, dst, n_mp};
  // rows are fetched one round ahead: the next round's start and length at
  // the top of a round, its node ids once this round's Newton solve is done,
  // so a round begins with its node gathers instead of two dependent loads
  // round k of chunk c (this workgroup's chunks are c_lo + j, + wgs, ...)
  auto row_at = [&](int64_t c, int64_t k, RowIds<PPL>& rw) {
    rw.off = 0;
    rw.end = 0;
    rw.K = 0;
    const int64_t i = k * per_round + tid / G;  // place in the chunk
    const int64_t q = c * chunk + i;
    if (ok && c < c_hi && i < chunk && q < n_mp) {
      rw.off = offsets[q];
      rw.end = offsets[q + 1];
    }
  };
  // the next round's ids are fetched once this round's Newton solve is done
  // and waited for together with the MP's own loads
  RowIds<PPL> cur, nxt;
  auto fetch = [&]() { load_row_ids<G, PPL>(nxt, idx, lane); };
  auto wait = [&]() { hold_row(nxt); };
  const MidHooks<decltype(fetch), decltype(wait)> mid{fetch, wait};
  int64_t c = c_lo + j, k = 0;
  row_at(c, 0, nxt);
  fetch();
  wait();
  cur = nxt;
  while (c < c_hi) {
    const int64_t i = k * per_round + tid / G;  // place in the chunk
    const int64_t p = c * chunk + i;
    const bool chunk_end = k + 1 == rpc;
    const int64_t cn = chunk_end ? c + wgs : c, kn = chunk_end ? 0 : k + 1;
    row_at(cn, kn, nxt);
    if (ok && i < chunk && p < n_mp) {
      if (cur.K <= G * PPL)
        lme_point<G, PPL, true, DN>(p, lane, ns, n_mp, xp, offsets, idx, cap, beta, tol,
                                    max_iter, lam, N, dN, diag, sink, &cur, mid);
      else
        lme_point<G, PPL, false, DN>(p, lane, ns, n_mp, xp, offsets, idx, cap, beta, tol,
                                     max_iter, lam, N, dN, diag, sink, &cur, mid);
    }
    // a lane without an MP this round (past its chunk's end, or past the last
    // MP) has an empty next row: the next round is further on in the same
    // chunk, or there is none (a chunk that ends early is the workgroup's
    // only one, or the last of all), so it fetches no ids
    cur = nxt;
    if (chunk_end || (k + 1) % kLmeAsmFlushRounds == 0) {
      __syncthreads();
      table_flush(table, tid, 256, dst);
      __syncthreads();
    }
    c = cn;
    k = kn;
  }
  __syncthreads();
  table_flush(table, tid, 256, dst);
}

void launch_lme(int64_t n_nodes, const double* x_nodes, int64_t n_mp, const double* x_mp,
                const int64_t* nbr_offsets, const int32_t* nbr_idx, int64_t pair_capacity,
                double beta, double tol, int32_t max_iter, double* lam, double* N, void* dN,
                int32_t precision, const double4* packed, otm_diag* diag, hipStream_t s,
                const AsmIn* fused, const SegIn* seg) {
  if (n_mp <= 0) return;
  const NodeSrc ns{x_nodes, packed, n_nodes};
  constexpr int G = 4, PPL = 9;
  if (fused != nullptr) {
    static_assert(256 / G == 64, "rounds of 64 MPs");
    const int64_t chunk = lme_asm_chunk(n_mp);
    auto run = [&](auto kernel, auto* dn) {
      kernel<<<kLmeAsmBlocks, 256, 0, s>>>(ns, n_mp, x_mp, nbr_offsets, nbr_idx, pair_capacity,
                                           beta, tol, max_iter, lam, N, dn, diag, *fused, chunk);
    };
    const bool heat = fused->heat != nullptr;
    if (precision == OTM_FP64) {
      if (heat) run(k_lme_asm<G, PPL, double, true, double>, (double*)dN);
      else run(k_lme_asm<G, PPL, double, false, double>, (double*)dN);
    } else if (precision == OTM_MIXED) {
      if (heat) run(k_lme_asm<G, PPL, float, true, float>, (float*)dN);
      else run(k_lme_asm<G, PPL, float, false, float>, (float*)dN);
    } else {
      if (heat) run(k_lme_asm<G, PPL, float, true, double>, (float*)dN);
      else run(k_lme_asm<G, PPL, float, false, double>, (float*)dN);
    }
    return;
  }
  const unsigned nb = (unsigned)((n_mp + (256 / G) - 1) / (256 / G));
  auto run = [&](auto sink, auto* dn) {
    k_lme<G, PPL><<<nb, 256, 0, s>>>(ns, n_mp, x_mp, nbr_offsets, nbr_idx, pair_capacity, beta,
                                     tol, max_iter, lam, N, dn, diag, sink);
  };
  if (precision == OTM_FP64) {
    if (seg != nullptr)
      run(SegSink<double, double>{seg->vol, seg->mass, (const double*)seg->sigma, seg->pos_of,
                                  seg->contrib, n_mp},
          (double*)dN);
    else
      run(NoSink{}, (double*)dN);
  } else if (seg != nullptr && precision == OTM_MIXED) {
    run(SegSink<float, float>{seg->vol, seg->mass, (const float*)seg->sigma, seg->pos_of,
                              seg->contrib, n_mp},
        (float*)dN);
  } else if (seg != nullptr) {
    run(SegSink<float, double>{seg->vol, seg->mass, (const float*)seg->sigma, seg->pos_of,
                               seg->contrib, n_mp},
        (float*)dN);
  } else {
    run(NoSink{}, (float*)dN);
  }
}

}  // namespace otm
