// Deterministic nodal assembly.  The influence domain of a node (the MPs
// whose support holds it) is the transpose of the support lists (Sec. 2.1):
// pairs are bucketed by node with a counting sort, each bucket is then put in
// ascending pair order, and every node sums its own contributions
//   m_I = sum_p N_Ip m_p,   f_I = -sum_p v_p sigma_p grad N_Ip
// in that fixed order, so the result is identical from run to run.
#include "launch.h"
#include "otm_common.h"

namespace otm {

// Stabilisation term of the nodal force (Sec. 2.1, stabilised residual):
// pair (p, I) adds -eps N_Ip e_Ip with the under-integration error
//   e_Ip = [(x_I - x_p) - (1 + H_p)(x_I,prev - x_p,prev)] / |x_I,prev - x_p,prev|,
// H_p = dF_p - 1 of this step's MP update, x_I,prev = x_I - du_I.  Float64 in
// both precisions (positions and their differences).
struct StabMP {
  double x[3], xq[3], H[9];
};

OTM_DEV void stab_load(const Stab& sb, int64_t n_mp, int64_t p, StabMP& m) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    m.x[c] = sb.xp[c * n_mp + p];
    m.xq[c] = sb.xp_prev[c * n_mp + p];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) m.H[k] = sb.dFm1[k * n_mp + p];
}

OTM_DEV void stab_add(const Stab& sb, const StabMP& m, int32_t I, double Nq, double& c1,
                      double& c2, double& c3) {
  const double2* __restrict__ nd = reinterpret_cast<const double2*>(sb.nodes);
  const double2 ra = nd[4 * (int64_t)I], rb = nd[4 * (int64_t)I + 1];
  const double2 rc = nd[4 * (int64_t)I + 2];
  const double xi[3] = {ra.x, ra.y, rb.x}, ui[3] = {rb.y, rc.x, rc.y};
  double d[3], dp[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d[k] = xi[k] - m.x[k];
    dp[k] = (xi[k] - ui[k]) - m.xq[k];
  }
  const double w = -sb.eps * Nq / sqrt((dp[0] * dp[0] + dp[1] * dp[1]) + dp[2] * dp[2]);
  double e[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
    e[i] = d[i] - (dp[i] + (m.H[3 * i] * dp[0] + m.H[3 * i + 1] * dp[1] + m.H[3 * i + 2] * dp[2]));
  c1 += w * e[0];
  c2 += w * e[1];
  c3 += w * e[2];
}

// Counting sort of the pairs by node.  A workgroup takes 512 consecutive MPs
// (rows walked by 8 lanes each), counts its pairs per node in an LDS hash
// table, and adds one global atomic per distinct node; the fill repeats the
// count, reserves each node's run with one global atomic, and places each
// pair at its rank inside the workgroup's run.  Bucket order is then fixed
// by k_tr_sort.
constexpr int kTrMPs = 512;
constexpr int kTrLanes = 8;
constexpr int kTrSlotBits = 11;
constexpr int kTrSlots = 1 << kTrSlotBits;

struct TrTable {
  int32_t key[kTrSlots];
  int32_t cnt[kTrSlots];
  int32_t base[kTrSlots];
};

OTM_DEV void tr_clear(TrTable& t) {
  for (int i = threadIdx.x; i < kTrSlots; i += blockDim.x) {
    t.key[i] = -1;
    t.cnt[i] = 0;
  }
}

// Slot of node I in the table (claimed if new), or -1 if the table is full.
OTM_DEV int tr_slot(TrTable& t, int32_t I) {
  uint32_t h = ((uint32_t)I * 2654435761u) >> (32 - kTrSlotBits);
  for (int probe = 0; probe < 64; ++probe) {
    const int32_t prev = atomicCAS(&t.key[h], -1, I);
    if (prev == -1 || prev == I) return (int)h;
    h = (h + 1) & (kTrSlots - 1);
  }
  return -1;
}

template <typename Visit>
OTM_DEV void tr_for_each_pair(int64_t base, int64_t n_mp, const int64_t* __restrict__ offsets,
                              Visit&& visit) {
  const int lane = threadIdx.x % kTrLanes;
  for (int r = 0; r < kTrMPs / (256 / kTrLanes); ++r) {
    const int64_t p = base + r * (256 / kTrLanes) + threadIdx.x / kTrLanes;
    if (p >= n_mp) continue;
    for (int64_t q = offsets[p] + lane; q < offsets[p + 1]; q += kTrLanes) visit(q);
  }
}

__global__ __launch_bounds__(256) void k_tr_count(int64_t n_mp, int64_t cap,
                                                  const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx,
                                                  unsigned long long* __restrict__ cnt) {
  __shared__ TrTable t;
  if (offsets[n_mp] > cap) return;  // lists were not written (capacity)
  tr_clear(t);
  __syncthreads();
  const int64_t base = (int64_t)xcd_block() * kTrMPs;
  tr_for_each_pair(base, n_mp, offsets, [&](int64_t q) {
    const int32_t I = idx[q];
    const int h = tr_slot(t, I);
    if (h >= 0) atomicAdd(&t.cnt[h], 1);
    else atomicAdd(&cnt[I + 1], 1ull);  // crowded table
  });
  __syncthreads();
  for (int i = threadIdx.x; i < kTrSlots; i += blockDim.x)
    if (t.key[i] >= 0) atomicAdd(&cnt[t.key[i] + 1], (unsigned long long)t.cnt[i]);
}

__global__ __launch_bounds__(256) void k_tr_fill(int64_t n_mp, int64_t cap,
                                                 const int64_t* __restrict__ offsets,
                                                 const int32_t* __restrict__ idx,
                                                 const int64_t* __restrict__ start,
                                                 int32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ pairs) {
  __shared__ TrTable t;
  if (offsets[n_mp] > cap) return;
  tr_clear(t);
  __syncthreads();
  const int64_t base = (int64_t)xcd_block() * kTrMPs;
  tr_for_each_pair(base, n_mp, offsets, [&](int64_t q) {
    const int h = tr_slot(t, idx[q]);
    if (h >= 0) atomicAdd(&t.cnt[h], 1);
  });
  __syncthreads();
  // reserve each node's run; the counters restart as ranks
  for (int i = threadIdx.x; i < kTrSlots; i += blockDim.x) {
    const int32_t I = t.key[i];
    if (I >= 0) {
      t.base[i] = (int32_t)start[I] + atomicAdd(&cursor[I], t.cnt[i]);
      t.cnt[i] = 0;
    }
  }
  __syncthreads();
  tr_for_each_pair(base, n_mp, offsets, [&](int64_t q) {
    const int32_t I = idx[q];
    const int h = tr_slot(t, I);  // finds the slot claimed above (or -1 if crowded)
    const int64_t pos = h >= 0 ? (int64_t)t.base[h] + atomicAdd(&t.cnt[h], 1)
                               : start[I] + atomicAdd(&cursor[I], 1);
    pairs[pos] = (int32_t)q;
  });
}

// Sixteen lanes per node: the bucket (distinct pair ids) put in ascending
// order by a bitonic network over 256 slots, lane l of the node's 16-lane row
// holding slots 16l .. 16l + 15 (past the bucket: INT32_MAX), and each pair's
// place in that order written straight to pos_of, so the sorted bucket itself
// is never stored.  Compare-exchanges between slots 16 or more apart pair a
// lane with lane l ^ 1, ^ 2, ^ 4 or ^ 8 of its row (DPP quad permutations, a
// swizzle, a row rotation by 8); the others stay in the lane.  Buckets past
// kSortCap (degenerate inputs) are ranked from global memory.
constexpr int kSortLanes = 16;
constexpr int kSortNodes = 256 / kSortLanes;
constexpr int kSortCap = 256;
constexpr int kSortPer = kSortCap / kSortLanes;

// Value of lane l ^ M of the same 16-lane row.
template <int M>
OTM_DEV int32_t row_xor(int32_t v) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8, "lane distance within a row");
  if constexpr (M == 1) return dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  else if constexpr (M == 2) return dpp_move<0x4E>(v);  // quad_perm [2,3,0,1]
  else if constexpr (M == 4) return __builtin_amdgcn_ds_swizzle(v, (4 << 10) | 0x1F);
  else return dpp_move<0x128>(v);  // row_ror:8
}

// One compare-exchange stage at distance J of the merge of width K.
template <int K, int J>
OTM_DEV void sort_stage(int32_t (&a)[kSortPer], int l) {
  if constexpr (J >= kSortPer) {
    constexpr int M = J / kSortPer;
    const bool lower = (l & M) == 0;
#pragma unroll
    for (int e = 0; e < kSortPer; ++e) {
      const int32_t w = row_xor<M>(a[e]);
      const int32_t lo = a[e] < w ? a[e] : w, hi = a[e] < w ? w : a[e];
      const bool up = ((kSortPer * l + e) & K) == 0;
      a[e] = lower == up ? lo : hi;
    }
  } else {
#pragma unroll
    for (int e = 0; e < kSortPer; ++e) {
      const int f = e ^ J;
      if (f > e) {
        const int32_t x = a[e], y = a[f];
        const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
        const bool up = ((kSortPer * l + e) & K) == 0;
        a[e] = up ? lo : hi;
        a[f] = up ? hi : lo;
      }
    }
  }
}

template <int K, int J>
OTM_DEV void sort_merge(int32_t (&a)[kSortPer], int l) {
  sort_stage<K, J>(a, l);
  if constexpr (J > 1) sort_merge<K, J / 2>(a, l);
}

template <int K>
OTM_DEV void sort_levels(int32_t (&a)[kSortPer], int l) {
  sort_merge<K, K / 2>(a, l);
  if constexpr (K < kSortCap) sort_levels<2 * K>(a, l);
}

__global__ __launch_bounds__(256) void k_tr_sort(int64_t n_nodes, const int64_t* __restrict__ start,
                                                 const int32_t* __restrict__ pairs,
                                                 int32_t* __restrict__ pos_of) {
  const int g = threadIdx.x / kSortLanes, lane = threadIdx.x % kSortLanes;
  const int64_t I = (int64_t)xcd_block() * kSortNodes + g;
  if (I >= n_nodes) return;  // whole row leaves together
  const int64_t s0 = start[I];
  const int n = (int)(start[I + 1] - s0);
  if (n <= kSortCap) {
    int32_t a[kSortPer];
#pragma unroll
    for (int e = 0; e < kSortPer; ++e) {
      const int i = kSortPer * lane + e;
      a[e] = i < n ? pairs[s0 + i] : INT32_MAX;
    }
    sort_levels<2>(a, lane);
#pragma unroll
    for (int e = 0; e < kSortPer; ++e) {
      const int i = kSortPer * lane + e;
      if (i < n) pos_of[a[e]] = (int32_t)(s0 + i);
    }
  } else {
    for (int i = lane; i < n; i += kSortLanes) {
      const int32_t v = pairs[s0 + i];
      int r = 0;
      for (int j = 0; j < n; ++j) r += pairs[s0 + j] < v;
      pos_of[v] = (int32_t)(s0 + r);
    }
  }
}

void launch_influence_lists(const otm_state& st, const Workspace& w, hipStream_t s) {
  const int64_t nn = st.n_nodes, nm = st.n_mp;
  if (nn <= 0) return;
  launch_fill_i64(w.tr_start, nn + 1, 0, s);
  launch_fill_i32(w.tr_cursor, nn, 0, s);
  if (nm > 0) {
    const unsigned nb = (unsigned)((nm + kTrMPs - 1) / kTrMPs);
    k_tr_count<<<nb, 256, 0, s>>>(nm, st.pair_capacity, st.nbr_offsets, st.nbr_idx,
                                  (unsigned long long*)w.tr_start);
    scan_inclusive(w.tr_start + 1, nn, w.scan_aux, s);
    k_tr_fill<<<nb, 256, 0, s>>>(nm, st.pair_capacity, st.nbr_offsets, st.nbr_idx, w.tr_start,
                                 w.tr_cursor, w.tr_pairs);
    k_tr_sort<<<(unsigned)((nn + kSortNodes - 1) / kSortNodes), 256, 0, s>>>(nn, w.tr_start,
                                                                             w.tr_pairs, w.tr_pos);
  }
}

// Deterministic assembly.  Per step, each pair's four contributions
// (N m_p and -v sigma grad N) are computed MP by MP and stored at the pair's
// place in the node-sorted order; each node then sums its contiguous run in
// that fixed order (ascending pair id) with a fixed reduction tree, so the
// result is identical from run to run and the gather reads are unit-stride.
constexpr int kScLanes = 8;
constexpr int kScMPs = 256 / kScLanes;

template <typename R, typename Q, bool STAB>
__global__ __launch_bounds__(256) void k_seg_contrib(
    int64_t n_mp, int64_t cap, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ idx, const double* __restrict__ N, const R* __restrict__ dN,
    const double* __restrict__ vol, const double* __restrict__ mass,
    const R* __restrict__ sigma, const int32_t* __restrict__ pos_of,
    double4* __restrict__ contrib, Stab sb) {
  const int64_t p = (int64_t)xcd_block() * kScMPs + threadIdx.x / kScLanes;
  const int lane = threadIdx.x % kScLanes;
  if (p >= n_mp) return;
  if (offsets[n_mp] > cap) return;
  const double mp = mass[p];
  const double v = vol[p];
  const R s0 = sigma[p], s1 = sigma[n_mp + p], s2 = sigma[2 * n_mp + p];
  const R s3 = sigma[3 * n_mp + p], s4 = sigma[4 * n_mp + p], s5 = sigma[5 * n_mp + p];
  StabMP sm;
  if constexpr (STAB) stab_load(sb, n_mp, p, sm);
  for (int64_t q = offsets[p] + lane; q < offsets[p + 1]; q += kScLanes) {
    const R g0 = dN[q], g1 = dN[cap + q], g2 = dN[2 * cap + q];
    const double Nq = N[q];
    double c1, c2, c3;
    pair_force<Q>(v, s0, s1, s2, s3, s4, s5, g0, g1, g2, c1, c2, c3);
    if constexpr (STAB) stab_add(sb, sm, idx[q], Nq, c1, c2, c3);
    contrib[pos_of[q]] = make_double4(Nq * mp, c1, c2, c3);
  }
}

constexpr int kSegLanes = 8;

__global__ __launch_bounds__(256) void k_seg_gather(int64_t n_nodes, int64_t n_mp, int64_t cap,
                                                    const int64_t* __restrict__ offsets,
                                                    const int64_t* __restrict__ start,
                                                    const double4* __restrict__ contrib,
                                                    double* __restrict__ m,
                                                    double* __restrict__ f) {
  const int64_t I = (int64_t)xcd_block() * (256 / kSegLanes) + threadIdx.x / kSegLanes;
  const int lane = threadIdx.x % kSegLanes;
  if (I >= n_nodes) return;
  if (offsets[n_mp] > cap) return;
  double am = 0, a0 = 0, a1 = 0, a2 = 0;
  for (int64_t j = start[I] + lane; j < start[I + 1]; j += kSegLanes) {
    const double4 c = contrib[j];
    am += c.x; a0 += c.y; a1 += c.z; a2 += c.w;
  }
  am = group_sum<kSegLanes>(am);
  a0 = group_sum<kSegLanes>(a0);
  a1 = group_sum<kSegLanes>(a1);
  a2 = group_sum<kSegLanes>(a2);
  if (lane == 0) {
    m[I] = am;
    f[I] = a0;
    f[n_nodes + I] = a1;
    f[2 * n_nodes + I] = a2;
  }
}

template <typename R, typename Q, bool STAB>
static void seg_contrib(const otm_state& st, const Workspace& w, const Stab& sb, hipStream_t s) {
  const int64_t nm = st.n_mp;
  const unsigned nb = (unsigned)((nm + kScMPs - 1) / kScMPs);
  k_seg_contrib<R, Q, STAB><<<nb, 256, 0, s>>>(nm, st.pair_capacity, st.nbr_offsets, st.nbr_idx,
                                            st.N, (const R*)st.dN, st.vol, st.mass,
                                            (const R*)st.sigma, w.tr_pos, w.contrib, sb);
}

void launch_scatter_segmented(const otm_state& st, const Workspace& w, const Stab& sb,
                              hipStream_t s) {
  const int64_t nn = st.n_nodes, nm = st.n_mp;
  if (nn <= 0) return;
  if (nm > 0) {
    const bool stab = sb.eps > 0.0;
    if (st.precision == OTM_FP64)
      stab ? seg_contrib<double, double, true>(st, w, sb, s)
           : seg_contrib<double, double, false>(st, w, sb, s);
    else if (st.precision == OTM_MIXED)
      stab ? seg_contrib<float, float, true>(st, w, sb, s)
           : seg_contrib<float, float, false>(st, w, sb, s);
    else
      stab ? seg_contrib<float, double, true>(st, w, sb, s)
           : seg_contrib<float, double, false>(st, w, sb, s);
  }
  launch_seg_gather(st, w, s);
}

void launch_seg_gather(const otm_state& st, const Workspace& w, hipStream_t s) {
  const int64_t nn = st.n_nodes;
  if (nn <= 0) return;
  const unsigned nb = (unsigned)((nn + (256 / kSegLanes) - 1) / (256 / kSegLanes));
  k_seg_gather<<<nb, 256, 0, s>>>(nn, st.n_mp, st.pair_capacity, st.nbr_offsets, w.tr_start,
                                  w.contrib, st.m, st.f);
}

}  // namespace otm

namespace otm {

// Atomic assembly with workgroup pre-aggregation.  A workgroup takes 512
// consecutive MPs (spatially compact, so they share most of their nodes),
// sums their contributions per node in an LDS table (NodeTable), then adds
// each distinct node's four sums to m and f with one float64 atomic each.
// Summation order varies from run to run.  Without the stabilisation term
// the step fuses this into the shape-function kernel instead (lme.hip).
constexpr int kAsmMPs = 512;
constexpr int kAsmLanes = 8;

template <typename R, typename Q, bool STAB>
__global__ __launch_bounds__(256) void k_assemble_atomic(
    int64_t n_nodes, int64_t n_mp, int64_t cap, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ idx, const double* __restrict__ N, const R* __restrict__ dN,
    const double* __restrict__ vol, const double* __restrict__ mass, const R* __restrict__ sigma,
    double* __restrict__ m, double* __restrict__ f, Stab sb) {
  __shared__ NodeTable table;
  const int tid = threadIdx.x;
  table_clear(table, tid, 256);
  __syncthreads();
  const bool ok = offsets[n_mp] <= cap;
  const int64_t base = (int64_t)xcd_block() * kAsmMPs;
  const int lane = tid % kAsmLanes;
  for (int r = 0; r < kAsmMPs / (256 / kAsmLanes); ++r) {
    const int64_t p = base + r * (256 / kAsmLanes) + tid / kAsmLanes;
    if (!ok || p >= n_mp) continue;
    const double mp = mass[p];
    const double v = vol[p];
    const R s0 = sigma[p], s1 = sigma[n_mp + p], s2 = sigma[2 * n_mp + p];
    const R s3 = sigma[3 * n_mp + p], s4 = sigma[4 * n_mp + p], s5 = sigma[5 * n_mp + p];
    const int64_t o0 = offsets[p], o1 = offsets[p + 1];
    if (o1 == o0) continue;
    StabMP sm;
    if constexpr (STAB) stab_load(sb, n_mp, p, sm);
    auto insert = [&](int32_t I, double c0, double c1, double c2, double c3) {
      table_insert(table, I, c0, c1, c2, c3, m, f, n_nodes);
    };
    auto contrib = [&](int64_t q, int32_t& I, double& c0, double& c1, double& c2, double& c3) {
      I = idx[q];
      const R g0 = dN[q], g1 = dN[cap + q], g2 = dN[2 * cap + q];
      const double Nq = N[q];
      c0 = Nq * mp;
      pair_force<Q>(v, s0, s1, s2, s3, s4, s5, g0, g1, g2, c1, c2, c3);
      if constexpr (STAB) stab_add(sb, sm, I, Nq, c1, c2, c3);
    };
    const int K = (int)(o1 - o0);
    auto slot = [&](int t) { return o0 + t; };
    // first 4 slots per lane: loads issued together (row start stands in for
    // slots past the end), then the table updates
    int32_t Iu[4];
    double cu[4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int t = k * kAsmLanes + lane;
      contrib(t < K ? slot(t) : o0, Iu[k], cu[k][0], cu[k][1], cu[k][2], cu[k][3]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k * kAsmLanes + lane < K) insert(Iu[k], cu[k][0], cu[k][1], cu[k][2], cu[k][3]);
    for (int t = 4 * kAsmLanes + lane; t < K; t += kAsmLanes) {
      int32_t I;
      double c0, c1, c2, c3;
      contrib(slot(t), I, c0, c1, c2, c3);
      insert(I, c0, c1, c2, c3);
    }
  }
  __syncthreads();
  table_flush(table, tid, 256, m, f, n_nodes);
}

template <typename R, typename Q, bool STAB>
static void assemble_atomic(const otm_state& st, const Stab& sb, hipStream_t s) {
  const int64_t nm = st.n_mp;
  const unsigned nb = (unsigned)((nm + kAsmMPs - 1) / kAsmMPs);
  k_assemble_atomic<R, Q, STAB><<<nb, 256, 0, s>>>(st.n_nodes, nm, st.pair_capacity,
                                                st.nbr_offsets, st.nbr_idx, st.N,
                                                (const R*)st.dN, st.vol, st.mass,
                                                (const R*)st.sigma, st.m, st.f, sb);
}

void launch_assemble_atomic(const otm_state& st, const Stab& sb, hipStream_t s) {
  if (st.n_mp <= 0) return;
  const bool stab = sb.eps > 0.0;
  if (st.precision == OTM_FP64)
    stab ? assemble_atomic<double, double, true>(st, sb, s)
         : assemble_atomic<double, double, false>(st, sb, s);
  else if (st.precision == OTM_MIXED)
    stab ? assemble_atomic<float, float, true>(st, sb, s)
         : assemble_atomic<float, float, false>(st, sb, s);
  else
    stab ? assemble_atomic<float, double, true>(st, sb, s)
         : assemble_atomic<float, double, false>(st, sb, s);
}

}  // namespace otm
