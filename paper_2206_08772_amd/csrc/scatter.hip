// Deterministic nodal assembly.  The influence domain of a node (the MPs
// whose support holds it) is the transpose of the support lists (Sec. 2.1):
// pairs are bucketed by node with a counting sort, each bucket is then put in
// ascending pair order, and every node sums its own contributions
//   m_I = sum_p N_Ip m_p,   f_I = -sum_p v_p sigma_p grad N_Ip
// in that fixed order, so the result is identical from run to run.
#include "launch.h"
#include "otm_common.h"

namespace otm {

__global__ __launch_bounds__(256) void k_tr_count(int64_t n_mp, int64_t cap,
                                                  const int64_t* __restrict__ offsets,
                                                  const int32_t* __restrict__ idx,
                                                  unsigned long long* __restrict__ cnt,
                                                  int32_t* __restrict__ pair_mp) {
  const int64_t p = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  if (p >= n_mp) return;
  if (offsets[n_mp] > cap) return;  // lists were not written (capacity)
  for (int64_t q = offsets[p]; q < offsets[p + 1]; ++q) {
    atomicAdd(&cnt[idx[q] + 1], 1ull);
    pair_mp[q] = (int32_t)p;
  }
}

__global__ __launch_bounds__(256) void k_tr_fill(int64_t n_mp, int64_t cap,
                                                 const int64_t* __restrict__ offsets,
                                                 const int32_t* __restrict__ idx,
                                                 const int64_t* __restrict__ start,
                                                 int32_t* __restrict__ cursor,
                                                 int32_t* __restrict__ pairs) {
  const int64_t p = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
  if (p >= n_mp) return;
  if (offsets[n_mp] > cap) return;
  for (int64_t q = offsets[p]; q < offsets[p + 1]; ++q) {
    const int32_t I = idx[q];
    const int32_t slot = atomicAdd(&cursor[I], 1);
    pairs[start[I] + slot] = (int32_t)q;
  }
}

// One wave per node: rank sort of the bucket (pair ids are distinct).
constexpr int kSortLds = 1024;
__global__ __launch_bounds__(256) void k_tr_sort(int64_t n_nodes, const int64_t* __restrict__ start,
                                                 int32_t* __restrict__ pairs) {
  __shared__ int32_t buf[4][kSortLds];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int64_t I = (int64_t)blockIdx.x * 4 + w;
  if (I >= n_nodes) return;
  const int64_t s0 = start[I];
  const int n = (int)(start[I + 1] - s0);
  if (n <= 1) return;
  if (n <= kSortLds) {
    for (int i = lane; i < n; i += kWave) buf[w][i] = pairs[s0 + i];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    int32_t vals[kSortLds / kWave];
    int ranks[kSortLds / kWave];
    int cntv = 0;
    for (int i = lane; i < n; i += kWave) {
      const int32_t v = buf[w][i];
      int r = 0;
      for (int j = 0; j < n; ++j) r += buf[w][j] < v;
      vals[cntv] = v;
      ranks[cntv] = r;
      ++cntv;
    }
    for (int k = 0; k < cntv; ++k) pairs[s0 + ranks[k]] = vals[k];
  } else if (lane == 0) {
    // very long bucket: insertion sort in place by one lane
    for (int i = 1; i < n; ++i) {
      const int32_t v = pairs[s0 + i];
      int j = i;
      while (j > 0 && pairs[s0 + j - 1] > v) {
        pairs[s0 + j] = pairs[s0 + j - 1];
        --j;
      }
      pairs[s0 + j] = v;
    }
  }
}

void launch_influence_lists(const otm_state& st, const Workspace& w, hipStream_t s) {
  const int64_t nn = st.n_nodes, nm = st.n_mp;
  if (nn <= 0) return;
  launch_fill_i64(w.tr_start, nn + 1, 0, s);
  launch_fill_i32(w.tr_cursor, nn, 0, s);
  if (nm > 0) {
    const unsigned nb = (unsigned)((nm + 255) / 256);
    k_tr_count<<<nb, 256, 0, s>>>(nm, st.pair_capacity, st.nbr_offsets, st.nbr_idx,
                                  (unsigned long long*)w.tr_start, w.pair_mp);
    scan_inclusive(w.tr_start + 1, nn, w.scan_aux, s);
    k_tr_fill<<<nb, 256, 0, s>>>(nm, st.pair_capacity, st.nbr_offsets, st.nbr_idx, w.tr_start, w.tr_cursor,
                                 w.tr_pairs);
    k_tr_sort<<<(unsigned)((nn + 3) / 4), 256, 0, s>>>(nn, w.tr_start, w.tr_pairs);
  }
}

constexpr int kSegLanes = 8;

template <typename R>
__global__ __launch_bounds__(256) void k_scatter_seg(
    int64_t n_nodes, int64_t n_mp, int64_t cap, const int64_t* __restrict__ offsets,
    const int64_t* __restrict__ start, const int32_t* __restrict__ pairs,
    const int32_t* __restrict__ pair_mp, const double* __restrict__ N, const R* __restrict__ dN,
    const double* __restrict__ vol, const double* __restrict__ mass,
    const R* __restrict__ sigma, double* __restrict__ m, double* __restrict__ f) {
  const int64_t I = (int64_t)xcd_block() * (256 / kSegLanes) + threadIdx.x / kSegLanes;
  const int lane = threadIdx.x % kSegLanes;
  if (I >= n_nodes) return;
  if (offsets[n_mp] > cap) return;
  double am = 0, a0 = 0, a1 = 0, a2 = 0;
  for (int64_t j = start[I] + lane; j < start[I + 1]; j += kSegLanes) {
    const int32_t q = pairs[j];
    const int32_t p = pair_mp[q];
    const double w = N[q];
    am += w * mass[p];
    const R g0 = dN[q], g1 = dN[cap + q], g2 = dN[2 * cap + q];
    const R s0 = sigma[p], s1 = sigma[n_mp + p], s2 = sigma[2 * n_mp + p];
    const R s3 = sigma[3 * n_mp + p], s4 = sigma[4 * n_mp + p], s5 = sigma[5 * n_mp + p];
    const R v = (R)vol[p];
    a0 += (double)(-v * (s0 * g0 + s3 * g1 + s5 * g2));
    a1 += (double)(-v * (s3 * g0 + s1 * g1 + s4 * g2));
    a2 += (double)(-v * (s5 * g0 + s4 * g1 + s2 * g2));
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

void launch_scatter_segmented(const otm_state& st, const Workspace& w, hipStream_t s) {
  const int64_t nn = st.n_nodes;
  if (nn <= 0) return;
  const unsigned nb = (unsigned)((nn + (256 / kSegLanes) - 1) / (256 / kSegLanes));
  if (st.precision == OTM_FP64)
    k_scatter_seg<double><<<nb, 256, 0, s>>>(nn, st.n_mp, st.pair_capacity, st.nbr_offsets,
                                             w.tr_start, w.tr_pairs, w.pair_mp, st.N,
                                             (const double*)st.dN, st.vol, st.mass,
                                             (const double*)st.sigma, st.m, st.f);
  else
    k_scatter_seg<float><<<nb, 256, 0, s>>>(nn, st.n_mp, st.pair_capacity, st.nbr_offsets,
                                            w.tr_start, w.tr_pairs, w.pair_mp, st.N,
                                            (const float*)st.dN, st.vol, st.mass,
                                            (const float*)st.sigma, st.m, st.f);
}

}  // namespace otm

namespace otm {

// Atomic assembly with workgroup pre-aggregation.  A workgroup takes 512
// consecutive MPs (spatially compact, so they share most of their nodes),
// sums their contributions per node in an LDS hash table (open addressing on
// the node id), then adds each distinct node's four sums to m and f with one
// float64 atomic each.  Summation order varies from run to run.
constexpr int kAsmMPs = 512;
constexpr int kAsmLanes = 8;
constexpr int kAsmSlotBits = 10;
constexpr int kAsmSlots = 1 << kAsmSlotBits;

template <typename R>
__global__ __launch_bounds__(256) void k_assemble_atomic(
    int64_t n_nodes, int64_t n_mp, int64_t cap, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ idx, const double* __restrict__ N, const R* __restrict__ dN,
    const double* __restrict__ vol, const double* __restrict__ mass, const R* __restrict__ sigma,
    double* __restrict__ m, double* __restrict__ f) {
  __shared__ int32_t keys[kAsmSlots];
  __shared__ double vals[4][kAsmSlots];
  const int tid = threadIdx.x;
  for (int s = tid; s < kAsmSlots; s += 256) {
    keys[s] = -1;
    vals[0][s] = vals[1][s] = vals[2][s] = vals[3][s] = 0.0;
  }
  __syncthreads();
  const bool ok = offsets[n_mp] <= cap;
  const int64_t base = (int64_t)xcd_block() * kAsmMPs;
  const int lane = tid % kAsmLanes;
  for (int r = 0; r < kAsmMPs / (256 / kAsmLanes); ++r) {
    const int64_t p = base + r * (256 / kAsmLanes) + tid / kAsmLanes;
    if (!ok || p >= n_mp) continue;
    const double mp = mass[p];
    const R v = (R)vol[p];
    const R s0 = sigma[p], s1 = sigma[n_mp + p], s2 = sigma[2 * n_mp + p];
    const R s3 = sigma[3 * n_mp + p], s4 = sigma[4 * n_mp + p], s5 = sigma[5 * n_mp + p];
    const int64_t o0 = offsets[p], o1 = offsets[p + 1];
    if (o1 == o0) continue;
    auto insert = [&](int32_t I, double c0, double c1, double c2, double c3) {
      uint32_t h = ((uint32_t)I * 2654435761u) >> (32 - kAsmSlotBits);
      int slot = -1;
      for (int probe = 0; probe < 32; ++probe) {
        const int32_t prev = atomicCAS(&keys[h], -1, I);
        if (prev == -1 || prev == I) { slot = (int)h; break; }
        h = (h + 1) & (kAsmSlots - 1);
      }
      if (slot >= 0) {
        atomicAdd(&vals[0][slot], c0);
        atomicAdd(&vals[1][slot], c1);
        atomicAdd(&vals[2][slot], c2);
        atomicAdd(&vals[3][slot], c3);
      } else {  // crowded table: straight to memory
        atomicAdd(&m[I], c0);
        atomicAdd(&f[I], c1);
        atomicAdd(&f[n_nodes + I], c2);
        atomicAdd(&f[2 * n_nodes + I], c3);
      }
    };
    auto contrib = [&](int64_t q, int32_t& I, double& c0, double& c1, double& c2, double& c3) {
      I = idx[q];
      const R g0 = dN[q], g1 = dN[cap + q], g2 = dN[2 * cap + q];
      c0 = N[q] * mp;
      c1 = (double)(-v * (s0 * g0 + s3 * g1 + s5 * g2));
      c2 = (double)(-v * (s3 * g0 + s1 * g1 + s4 * g2));
      c3 = (double)(-v * (s5 * g0 + s4 * g1 + s2 * g2));
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
  for (int s = tid; s < kAsmSlots; s += 256) {
    const int32_t I = keys[s];
    if (I < 0) continue;
    atomicAdd(&m[I], vals[0][s]);
    atomicAdd(&f[I], vals[1][s]);
    atomicAdd(&f[n_nodes + I], vals[2][s]);
    atomicAdd(&f[2 * n_nodes + I], vals[3][s]);
  }
}

void launch_assemble_atomic(const otm_state& st, hipStream_t s) {
  const int64_t nm = st.n_mp;
  if (nm <= 0) return;
  const unsigned nb = (unsigned)((nm + kAsmMPs - 1) / kAsmMPs);
  if (st.precision == OTM_FP64)
    k_assemble_atomic<double><<<nb, 256, 0, s>>>(st.n_nodes, nm, st.pair_capacity,
                                                 st.nbr_offsets, st.nbr_idx, st.N,
                                                 (const double*)st.dN, st.vol, st.mass,
                                                 (const double*)st.sigma, st.m, st.f);
  else
    k_assemble_atomic<float><<<nb, 256, 0, s>>>(st.n_nodes, nm, st.pair_capacity,
                                                st.nbr_offsets, st.nbr_idx, st.N,
                                                (const float*)st.dN, st.vol, st.mass,
                                                (const float*)st.sigma, st.m, st.f);
}

}  // namespace otm
