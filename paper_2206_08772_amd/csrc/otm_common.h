// Device helpers shared by the OTM kernels: failure record, wave-level
// reductions, XCD-aware block numbering and small 3x3 tensor algebra.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "otm.h"

#define OTM_DEV __device__ __forceinline__
#define OTM_HD __host__ __device__ __forceinline__

namespace otm {

constexpr int kWave = 64;

// ----------------------------------------------------------------- failures
// Flag bit k corresponds to status -(k+1); counts and first indices are kept
// for the MP-level failures.
OTM_DEV void diag_fail(otm_diag* d, otm_status code, uint64_t index) {
  if (d == nullptr) return;
  const int k = -code - 1;
  atomicOr(&d->flags, 1u << k);
  unsigned long long* cnt = nullptr;
  unsigned long long* first = nullptr;
  switch (code) {
    case OTM_ERR_LME_NOCONV:
      cnt = (unsigned long long*)&d->n_lme_noconv;
      first = (unsigned long long*)&d->first_lme_noconv;
      break;
    case OTM_ERR_RM_NOCONV:
      cnt = (unsigned long long*)&d->n_rm_noconv;
      first = (unsigned long long*)&d->first_rm_noconv;
      break;
    case OTM_ERR_INVERTED:
      cnt = (unsigned long long*)&d->n_inverted;
      first = (unsigned long long*)&d->first_inverted;
      break;
    case OTM_ERR_NONFINITE:
      cnt = (unsigned long long*)&d->n_nonfinite;
      first = (unsigned long long*)&d->first_nonfinite;
      break;
    default:
      return;
  }
  atomicAdd(cnt, 1ull);
  atomicMin(first, (unsigned long long)index);
}

// ----------------------------------------------------------- block numbering
// The hardware deals consecutive workgroups round-robin to the 8 XCDs, each
// with its own L2.  Renumber so that every XCD works on one contiguous range
// of logical blocks (neighbouring MPs share nodes, so their gathers then hit
// the same L2).  Bijective on [0, gridDim.x).
OTM_DEV uint32_t xcd_block() {
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const uint32_t q = nb / 8u, r = nb % 8u, x = b % 8u;
  return x * q + (x < r ? x : r) + b / 8u;
}

// ------------------------------------------------------------ hold
// An empty statement that reads a loaded value.  Values loaded together and
// then used inside several branches (one per pair slot) are waited for once,
// at this point in straight-line code: otherwise the compiler moves a load
// used by one branch into that branch (its latency no longer overlaps the
// others), or waits at the top of every branch with a full wait, which also
// waits for every store issued before.
OTM_DEV void hold(double v) { __asm__ volatile("" ::"v"(v)); }
OTM_DEV void hold(float v) { __asm__ volatile("" ::"v"(v)); }
OTM_DEV void hold(int32_t v) { __asm__ volatile("" ::"v"(v)); }
OTM_DEV void hold(const double2& v) { hold(v.x); hold(v.y); }
OTM_DEV void hold(const double4& v) { hold(v.x); hold(v.y); hold(v.z); hold(v.w); }

// -------------------------------------------------------- pair force
// Internal-force contribution -v sigma grad N_Ip of one pair (the nodal
// residual, Sec. 2.1), sigma in Voigt order (xx yy zz xy yz xz).  sigma and
// grad N come in their stored type R; the products and sums are formed in
// Q (float32 in OTM_MIXED, float64 in the other modes) and handed on as
// float64 for the nodal accumulation.
template <typename Q, typename R>
OTM_DEV void pair_force(double v, R s0, R s1, R s2, R s3, R s4, R s5, R g0, R g1, R g2,
                        double& c1, double& c2, double& c3) {
  const Q h0 = g0, h1 = g1, h2 = g2;
  const Q t0 = s0, t1 = s1, t2 = s2, t3 = s3, t4 = s4, t5 = s5;
  const Q vq = (Q)v;
  c1 = (double)(-vq * (t0 * h0 + t3 * h1 + t5 * h2));
  c2 = (double)(-vq * (t3 * h0 + t1 * h1 + t4 * h2));
  c3 = (double)(-vq * (t5 * h0 + t4 * h1 + t2 * h2));
}

// ------------------------------------------------------------- reductions
// All-reduce over aligned groups of G <= 16 lanes with DPP row moves (no LDS
// round trip): row_ror:8 folds the two halves of a 16-lane row, then
// row_half_mirror, quad_perm [2,3,0,1] and quad_perm [1,0,3,2] finish the
// 8-lane groups.  Each stage adds a value to one that holds the same set of
// terms, so every lane of the group ends with the same bits (a + b and b + a
// round identically).
template <int CTRL, typename T>
OTM_DEV T dpp_move(T v) {
  return __builtin_amdgcn_update_dpp(T(0), v, CTRL, 0xF, 0xF, false);
}
template <int G, typename T, typename Op>
OTM_DEV T group_reduce(T v, Op op) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if constexpr (G >= 16) v = op(v, dpp_move<0x128>(v));  // row_ror:8
  if constexpr (G >= 8) v = op(v, dpp_move<0x141>(v));   // row_half_mirror
  if constexpr (G >= 4) v = op(v, dpp_move<0x4E>(v));    // quad_perm [2,3,0,1]
  if constexpr (G >= 2) v = op(v, dpp_move<0xB1>(v));    // quad_perm [1,0,3,2]
  return v;
}
template <int G, typename T>
OTM_DEV T group_sum(T v) {
  return group_reduce<G>(v, [](T a, T b) { return a + b; });
}

// One stage of row_sum_scatter: the lane keeps the lower or the upper half
// of its N-list (``upper``), sends the other half to its partner (the lane
// that keeps the opposite half of the same list) and adds what the partner
// sends.  A missing upper element (N odd) is a zero that stays zero.
template <int CTRL, int N, int M>
OTM_DEV void split_stage(const double (&in)[N], double (&out)[M], bool upper) {
  static_assert(M == (N + 1) / 2, "halving stage");
#pragma unroll
  for (int i = 0; i < M; ++i) {
    const double lo = in[i];
    const double hi = i + M < N ? in[i + M] : 0.0;
    out[i] = (upper ? hi : lo) + dpp_move<CTRL>(upper ? lo : hi);
  }
}

// Reduce-scatter over an aligned 16-lane row: V <= 16 values per lane in,
// the row's total of one of them out.  The four stages pair lane l with
// l ^ 8 (row_ror:8), then l ^ 7 (row_half_mirror), l ^ 2 and l ^ 1 (quad
// permutations); at each one the partners differ in the bit that picks the
// half kept (bits 3, 2, 1, 0) and agree in the bits of the earlier stages,
// so they hold the same list, and each lane's total collects all 16 lanes.
// The adds number about V instead of 4 V for V all-reduces.  ``c`` gets the
// index of the value whose total the lane holds, or -1 (a padding slot).
template <int V>
OTM_DEV double row_sum_scatter(const double (&a)[V], int& c) {
  static_assert(V >= 2 && V <= 16, "2 to 16 values over a 16-lane row");
  constexpr int M1 = (V + 1) / 2, M2 = (M1 + 1) / 2, M3 = (M2 + 1) / 2;
  static_assert((M3 + 1) / 2 == 1, "four stages");
  const int l = (int)(__lane_id() & 15u);
  double b1[M1], b2[M2], b3[M3], b4[1];
  split_stage<0x128>(a, b1, (l & 8) != 0);   // row_ror:8
  split_stage<0x141>(b1, b2, (l & 4) != 0);  // row_half_mirror
  split_stage<0x4E>(b2, b3, (l & 2) != 0);   // quad_perm [2,3,0,1]
  split_stage<0xB1>(b3, b4, (l & 1) != 0);   // quad_perm [1,0,3,2]
  // the kept element's place in the original list and whether it is real
  int idx = 0, len = V;
  auto step = [&](int m, bool upper) {
    if (upper) { idx += m; len -= m; } else if (len > m) { len = m; }
  };
  step(M1, (l & 8) != 0);
  step(M2, (l & 4) != 0);
  step(M3, (l & 2) != 0);
  step(1, (l & 1) != 0);
  c = len >= 1 ? idx : -1;
  return b4[0];
}
template <int G>
OTM_DEV double group_max(double v) {
  return group_reduce<G>(v, [](double a, double b) { return fmax(a, b); });
}

// Active lanes of a wave that count into the same slot share one atomic: the
// lanes of each distinct slot id are found by ballot (a wave-uniform loop of
// register operations only), then the lowest lane of every id adds its
// group's size, all ids in one atomic instruction (no chain of returning
// atomics), and each lane takes the value its group's atomic returned plus
// its rank in the group.  Spatially ordered items (lattice nodes, MPs in hex
// order) put few distinct slots in a wave.
template <typename C>
OTM_DEV C grouped_atomic_add(C* counters, int32_t cid) {
  const int lane = (int)__lane_id();
  uint64_t todo = __ballot(true);
  int leader = lane;
  C rank = 0, count = 0;
  while (todo) {
    const int l = __builtin_ctzll(todo);
    const int32_t lc = __builtin_amdgcn_readlane(cid, l);
    const uint64_t same = __ballot(cid == lc);
    if (cid == lc) {
      leader = l;
      rank = (C)__builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
    }
    if (lane == l) count = (C)__popcll(same);
    todo &= ~same;
  }
  C base = 0;
  if (lane == leader) base = atomicAdd(&counters[cid], count);
  return __shfl(base, leader) + rank;
}

// ------------------------------------------------------------- 3x3 algebra
template <typename R>
struct M3 {
  R a[3][3];
};
template <typename R>
struct S3 {  // symmetric: xx yy zz xy yz xz
  R v[6];
};

template <typename R>
OTM_HD R det3(const M3<R>& A) {
  return A.a[0][0] * (A.a[1][1] * A.a[2][2] - A.a[1][2] * A.a[2][1]) -
         A.a[0][1] * (A.a[1][0] * A.a[2][2] - A.a[1][2] * A.a[2][0]) +
         A.a[0][2] * (A.a[1][0] * A.a[2][1] - A.a[1][1] * A.a[2][0]);
}

// det(1 + X) - 1 = tr X + (tr^2 X - tr X^2)/2 + det X, accurate for small X.
template <typename R>
OTM_HD R det_one_plus_minus_one(const M3<R>& X) {
  const R tr = X.a[0][0] + X.a[1][1] + X.a[2][2];
  const R i2 = X.a[0][0] * X.a[1][1] + X.a[1][1] * X.a[2][2] + X.a[0][0] * X.a[2][2] -
               X.a[0][1] * X.a[1][0] - X.a[1][2] * X.a[2][1] - X.a[0][2] * X.a[2][0];
  return tr + i2 + det3(X);
}

// Symmetric 3x3 from its 6 components, as a full matrix.
template <typename R>
OTM_HD M3<R> full(const S3<R>& s) {
  M3<R> A;
  A.a[0][0] = s.v[0]; A.a[1][1] = s.v[1]; A.a[2][2] = s.v[2];
  A.a[0][1] = A.a[1][0] = s.v[3];
  A.a[1][2] = A.a[2][1] = s.v[4];
  A.a[0][2] = A.a[2][0] = s.v[5];
  return A;
}

// Eigen-decomposition of a symmetric 3x3 by cyclic Jacobi rotations:
// on return d[k] are the eigenvalues and column k of V the eigenvectors.
template <typename R>
OTM_HD void jacobi_eig(const S3<R>& s, R d[3], R V[3][3]) {
  R a00 = s.v[0], a11 = s.v[1], a22 = s.v[2];
  R a01 = s.v[3], a12 = s.v[4], a02 = s.v[5];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? R(1) : R(0);
  const R tiny = sizeof(R) == 8 ? R(1e-300) : R(1e-36);
  for (int sweep = 0; sweep < 12; ++sweep) {
    const R off = fabs(a01) + fabs(a12) + fabs(a02);
    const R diag = fabs(a00) + fabs(a11) + fabs(a22);
    if (off <= (sizeof(R) == 8 ? R(1e-18) : R(1e-9)) * diag || off < tiny) break;
    // rotation in plane (p, q); the three planes in turn
#pragma unroll
    for (int plane = 0; plane < 3; ++plane) {
      R app, aqq, apq;
      if (plane == 0) { app = a00; aqq = a11; apq = a01; }
      else if (plane == 1) { app = a00; aqq = a22; apq = a02; }
      else { app = a11; aqq = a22; apq = a12; }
      if (fabs(apq) < tiny) continue;
      const R theta = (aqq - app) / (R(2) * apq);
      const R t = (theta >= R(0) ? R(1) : R(-1)) / (fabs(theta) + sqrt(theta * theta + R(1)));
      const R c = R(1) / sqrt(t * t + R(1));
      const R sn = t * c;
      const R np = app - t * apq, nq = aqq + t * apq;
      if (plane == 0) {
        const R r02 = c * a02 - sn * a12, r12 = sn * a02 + c * a12;
        a00 = np; a11 = nq; a01 = R(0); a02 = r02; a12 = r12;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const R vp = V[k][0], vq = V[k][1];
          V[k][0] = c * vp - sn * vq; V[k][1] = sn * vp + c * vq;
        }
      } else if (plane == 1) {
        const R r01 = c * a01 - sn * a12, r21 = sn * a01 + c * a12;
        a00 = np; a22 = nq; a02 = R(0); a01 = r01; a12 = r21;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const R vp = V[k][0], vq = V[k][2];
          V[k][0] = c * vp - sn * vq; V[k][2] = sn * vp + c * vq;
        }
      } else {
        const R r10 = c * a01 - sn * a02, r20 = sn * a01 + c * a02;
        a11 = np; a22 = nq; a12 = R(0); a01 = r10; a02 = r20;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const R vp = V[k][1], vq = V[k][2];
          V[k][1] = c * vp - sn * vq; V[k][2] = sn * vp + c * vq;
        }
      }
    }
  }
  d[0] = a00; d[1] = a11; d[2] = a22;
}

// Q diag(w) Q^T as 6 components.
template <typename R>
OTM_HD S3<R> spectral_compose(const R V[3][3], const R w[3]) {
  S3<R> s;
  const int ii[6] = {0, 1, 2, 0, 1, 0}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const int i = ii[c], j = jj[c];
    s.v[c] = V[i][0] * w[0] * V[j][0] + V[i][1] * w[1] * V[j][1] + V[i][2] * w[2] * V[j][2];
  }
  return s;
}

// Inverse of a symmetric positive definite 3x3 given as xx yy zz xy yz xz.
OTM_HD void sym_inv(const double J[6], double Mi[6], double& det) {
  const double c00 = J[1] * J[2] - J[4] * J[4];
  const double c11 = J[0] * J[2] - J[5] * J[5];
  const double c22 = J[0] * J[1] - J[3] * J[3];
  const double c01 = J[5] * J[4] - J[3] * J[2];
  const double c12 = J[3] * J[5] - J[0] * J[4];
  const double c02 = J[3] * J[4] - J[5] * J[1];
  det = J[0] * c00 + J[3] * c01 + J[5] * c02;
  const double id = 1.0 / det;
  Mi[0] = c00 * id; Mi[1] = c11 * id; Mi[2] = c22 * id;
  Mi[3] = c01 * id; Mi[4] = c12 * id; Mi[5] = c02 * id;
}

OTM_HD void sym_mul_vec(const double M[6], const double v[3], double o[3]) {
  o[0] = M[0] * v[0] + M[3] * v[1] + M[5] * v[2];
  o[1] = M[3] * v[0] + M[1] * v[1] + M[4] * v[2];
  o[2] = M[5] * v[0] + M[4] * v[1] + M[2] * v[2];
}

// ------------------------------------------------ nodal assembly table
// A workgroup's per-node sums of V values (m and f, plus the two heat sums
// with conduction) in LDS: open addressing on the node id (multiplicative
// hash, linear probing).  A pair whose node finds no slot within 32 probes
// goes straight to memory with float64 atomics; flush adds each occupied
// slot's sums to their destination arrays with one atomic each and clears
// the table.  Summation order varies from run to run.
constexpr int kTableBits = 10;
constexpr int kTableSlots = 1 << kTableBits;

template <int V>
struct NodeTableV {
  int32_t keys[kTableSlots];
  double vals[V][kTableSlots];
};
using NodeTable = NodeTableV<4>;

// Destination arrays of a table's V sums, each indexed by node.
template <int V>
struct NodeDst {
  double* d[V];
};
OTM_HD NodeDst<4> mf_dst(double* m, double* f, int64_t n_nodes) {
  return NodeDst<4>{{m, f, f + n_nodes, f + 2 * n_nodes}};
}

template <int V>
OTM_DEV void table_clear(NodeTableV<V>& t, int tid, int nthreads) {
  for (int s = tid; s < kTableSlots; s += nthreads) {
    t.keys[s] = -1;
#pragma unroll
    for (int k = 0; k < V; ++k) t.vals[k][s] = 0.0;
  }
}

// Insertion of NB items per lane at once: every item's first probe (a
// compare-and-swap on its hash slot) is issued before any result is
// examined, so the LDS round trips overlap; an item whose slot holds another
// node probes on, one slot at a time (rare at the table's load).  Items with
// use[k] false are skipped.  The sums are the same as NB table_insert calls.
template <int V, int NB>
OTM_DEV void table_insert_batch(NodeTableV<V>& t, const int32_t (&I)[NB], const bool (&use)[NB],
                                const double (&c)[NB][V], const NodeDst<V>& dst) {
  uint32_t h[NB];
  int32_t prev[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    h[k] = ((uint32_t)I[k] * 2654435761u) >> (32 - kTableBits);
    prev[k] = use[k] ? atomicCAS(&t.keys[h[k]], -1, I[k]) : -1;
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (!use[k]) continue;
    int slot = -1;
    if (prev[k] == -1 || prev[k] == I[k]) {
      slot = (int)h[k];
    } else {
#pragma unroll 1
      for (int probe = 1; probe < 32; ++probe) {
        const uint32_t hh = (h[k] + (uint32_t)probe) & (kTableSlots - 1);
        const int32_t pv = atomicCAS(&t.keys[hh], -1, I[k]);
        if (pv == -1 || pv == I[k]) { slot = (int)hh; break; }
      }
    }
    if (slot >= 0) {
#pragma unroll
      for (int v = 0; v < V; ++v) atomicAdd(&t.vals[v][slot], c[k][v]);
    } else {  // crowded table: straight to memory
#pragma unroll
      for (int v = 0; v < V; ++v) atomicAdd(&dst.d[v][I[k]], c[k][v]);
    }
  }
}

template <int V>
OTM_DEV void table_insert(NodeTableV<V>& t, int32_t I, const double (&c)[V],
                          const NodeDst<V>& dst) {
  const int32_t key[1] = {I};
  const bool use[1] = {true};
  double cc[1][V];
#pragma unroll
  for (int v = 0; v < V; ++v) cc[0][v] = c[v];
  table_insert_batch<V, 1>(t, key, use, cc, dst);
}

OTM_DEV void table_insert(NodeTable& t, int32_t I, double c0, double c1, double c2, double c3,
                          double* m, double* f, int64_t n_nodes) {
  const double c[4] = {c0, c1, c2, c3};
  table_insert<4>(t, I, c, mf_dst(m, f, n_nodes));
}

// Every lane of the workgroup calls this after a barrier; it ends cleared
// (a barrier is needed before the next inserts).
template <int V>
OTM_DEV void table_flush(NodeTableV<V>& t, int tid, int nthreads, const NodeDst<V>& dst) {
  for (int s = tid; s < kTableSlots; s += nthreads) {
    const int32_t I = t.keys[s];
    if (I < 0) continue;
#pragma unroll
    for (int k = 0; k < V; ++k) {
      atomicAdd(&dst.d[k][I], t.vals[k][s]);
      t.vals[k][s] = 0.0;
    }
    t.keys[s] = -1;
  }
}

OTM_DEV void table_flush(NodeTable& t, int tid, int nthreads, double* m, double* f,
                         int64_t n_nodes) {
  table_flush<4>(t, tid, nthreads, mf_dst(m, f, n_nodes));
}

}  // namespace otm
