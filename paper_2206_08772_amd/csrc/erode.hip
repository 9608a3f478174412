// Removal of failed material points from the body: a stable stream
// compaction of every per-MP array of the state, for otm_erode.
#include <hip/hip_runtime.h>

#include "erode.h"
#include "otm_common.h"

namespace otm {

// ------------------------------------------------------------- erosion
// Removal of failed MPs from the body: a stable stream compaction of every
// per-MP array.  keep[p] = 1 for a surviving MP; its inclusive prefix sum is
// the survivor's new index + 1.
__global__ void k_keep_flags(int64_t n, const int32_t* __restrict__ failed,
                             int32_t* __restrict__ keep) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) keep[p] = failed[p] == 0 ? 1 : 0;
}

// Component-major [ncomp][n] -> [ncomp][n_keep], survivors in their order.
// One thread per MP: the reads are coalesced and the writes of a wave land
// in one contiguous run per component.
template <typename T>
__global__ void k_compact_field(const T* __restrict__ src, T* __restrict__ dst, int64_t n,
                                int64_t n_keep, int ncomp, const int32_t* __restrict__ pos,
                                const int32_t* __restrict__ failed) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || failed[p] != 0) return;
  const int64_t q = pos[p] - 1;
  for (int c = 0; c < ncomp; ++c) dst[c * n_keep + q] = src[c * n + p];
}

static_assert(sizeof(int32_t) * kRowCapacity >= sizeof(double) * 9,
              "the staging rows hold the widest per-MP field");

template <typename T>
static otm_status compact_field(T* a, int ncomp, int64_t n, int64_t n_keep,
                                const int32_t* failed, const Workspace& w, hipStream_t s) {
  T* tmp = reinterpret_cast<T*>(w.stage);
  const unsigned nb = (unsigned)((n + 255) / 256);
  k_compact_field<T><<<nb, 256, 0, s>>>(a, tmp, n, n_keep, ncomp, w.mp_cell, failed);
  if (hipGetLastError() != hipSuccess) return OTM_ERR_HIP;
  if (n_keep == 0) return OTM_OK;
  return hipMemcpyAsync(a, tmp, sizeof(T) * (size_t)ncomp * (size_t)n_keep,
                        hipMemcpyDeviceToDevice, s) == hipSuccess ? OTM_OK : OTM_ERR_HIP;
}

// ------------------------------------------ nodes added at the freed surface
// The removed MPs in ascending order: with keep_scan the inclusive prefix sum
// of the keep flags, MP p (removed) is the (p - keep_scan[p])-th removed one.
__global__ void k_removed_list(int64_t n, const int32_t* __restrict__ keep_scan,
                               int32_t* __restrict__ removed) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int32_t before = p > 0 ? keep_scan[p - 1] : 0;
  if (keep_scan[p] == before) removed[p - keep_scan[p]] = (int32_t)p;
}

OTM_DEV double erode_sqdist(double ax, double ay, double az, double bx, double by, double bz) {
#pragma clang fp contract(off)
  const double dx = ax - bx, dy = ay - by, dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

OTM_DEV double erode_madd(double a, double b, double c) {
#pragma clang fp contract(off)
  return a + b * c;
}

// One thread per removed MP (k-th): a node goes to x_p when every node of
// its support is farther than delta and no removed MP of smaller index lies
// within delta; it takes sum_I N_Ip du_I.  flag[k] = 1 for such MPs, and
// cand[c * n_rem + k] holds (x, y, z, du_x, du_y, du_z).  The check against
// the earlier removed MPs is a plain loop (cost quadratic in the removed
// count of one call).
__global__ void k_insert_candidates(int64_t n_rem, const int32_t* __restrict__ removed,
                                    const double* __restrict__ xp, int64_t n_mp,
                                    const double* __restrict__ x, const double* __restrict__ du,
                                    int64_t n_nodes, const int64_t* __restrict__ off,
                                    const int32_t* __restrict__ idx,
                                    const double* __restrict__ N, double d2,
                                    int32_t* __restrict__ flag, double* __restrict__ cand) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_rem) return;
  const int64_t p = removed[k];
  const double px = xp[p], py = xp[n_mp + p], pz = xp[2 * n_mp + p];
  bool ok = true;
  double u0 = 0.0, u1 = 0.0, u2 = 0.0;
  for (int64_t q = off[p]; q < off[p + 1]; ++q) {
    const int32_t I = idx[q];
    ok = ok && erode_sqdist(px, py, pz, x[I], x[n_nodes + I], x[2 * n_nodes + I]) > d2;
    // the interpolated increment in pair order, each product and sum
    // rounded on its own
    const double w = N[q];
    u0 = erode_madd(u0, w, du[I]);
    u1 = erode_madd(u1, w, du[n_nodes + I]);
    u2 = erode_madd(u2, w, du[2 * n_nodes + I]);
  }
  for (int64_t j = 0; ok && j < k; ++j) {
    const int64_t r = removed[j];
    ok = erode_sqdist(px, py, pz, xp[r], xp[n_mp + r], xp[2 * n_mp + r]) > d2;
  }
  flag[k] = ok ? 1 : 0;
  const double v[6] = {px, py, pz, u0, u1, u2};
  for (int c = 0; c < 6; ++c) cand[c * n_rem + k] = v[c];
}

// [ncomp][n] -> [ncomp][n_new] (n_new >= n) through a staging copy.
__global__ void k_restride(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                           int64_t n_new, int ncomp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < ncomp; ++c) dst[c * n_new + i] = src[c * n + i];
}

// The accepted candidates become nodes n .. n + k_ins - 1 (their order).
__global__ void k_place_nodes(int64_t n_rem, const int32_t* __restrict__ flag_scan,
                              const double* __restrict__ cand, int64_t n, int64_t n_new,
                              double* __restrict__ x, double* __restrict__ du,
                              double* __restrict__ gt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_rem) return;
  const int32_t before = k > 0 ? flag_scan[k - 1] : 0;
  if (flag_scan[k] == before) return;
  const int64_t I = n + before;
  for (int c = 0; c < 3; ++c) {
    x[c * n_new + I] = cand[c * n_rem + k];
    du[c * n_new + I] = cand[(3 + c) * n_rem + k];
    if (gt != nullptr) gt[c * n_new + I] = 0.0;
  }
}

static otm_status restride(double* a, int ncomp, int64_t n, int64_t n_new, double* tmp,
                           hipStream_t s) {
  if (n == 0) return OTM_OK;
  if (hipMemcpyAsync(tmp, a, sizeof(double) * (size_t)ncomp * (size_t)n,
                     hipMemcpyDeviceToDevice, s) != hipSuccess)
    return OTM_ERR_HIP;
  k_restride<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(tmp, a, n, n_new, ncomp);
  return hipGetLastError() == hipSuccess ? OTM_OK : OTM_ERR_HIP;
}

static otm_status insert_nodes(otm_state& st, const otm_params& p, int64_t n_rem,
                               const Workspace& w, int64_t* inserted, hipStream_t s) {
  *inserted = 0;
  const int64_t n_mp = st.n_mp, n = st.n_nodes;
  // staging in the search rows: removed list, flags, six candidate values
  int32_t* removed = w.stage;
  int32_t* flag = w.stage + n_mp;
  double* cand = reinterpret_cast<double*>(w.stage + 2 * n_mp + (n_mp & 1));
  k_removed_list<<<(unsigned)((n_mp + 255) / 256), 256, 0, s>>>(n_mp, w.mp_cell, removed);
  k_insert_candidates<<<(unsigned)((n_rem + 255) / 256), 256, 0, s>>>(
      n_rem, removed, st.xp, n_mp, st.x, st.du, n, st.nbr_offsets, st.nbr_idx, st.N,
      p.insert_dist * p.insert_dist, flag, cand);
  scan_inclusive(flag, n_rem, w.scan_aux, s);
  int32_t k_ins = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&k_ins, flag + (n_rem - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return OTM_ERR_HIP;
  if (k_ins == 0) return OTM_OK;
  const int64_t n_new = n + k_ins;
  const int64_t cap_nodes = st.node_capacity > n ? st.node_capacity : n;
  if (n_new > cap_nodes) return OTM_ERR_CAPACITY;
  if ((size_t)3 * (size_t)n * sizeof(double) > (size_t)st.pair_capacity * sizeof(double4))
    return OTM_ERR_ARG;  // no room to stage the node arrays (a state without pairs)
  double* tmp = reinterpret_cast<double*>(w.contrib);
  otm_status e = OTM_OK;
  auto run = [&](otm_status r) { if (e == OTM_OK) e = r; };
  run(restride(st.x, 3, n, n_new, tmp, s));
  run(restride(st.du, 3, n, n_new, tmp, s));
  double* gt = p.tool_enabled ? st.tool_gt : nullptr;
  if (gt != nullptr) run(restride(gt, 3, n, n_new, tmp, s));
  if (e != OTM_OK) return e;
  // m, f and the heat sums are assembled anew by the refresh
  k_place_nodes<<<(unsigned)((n_rem + 255) / 256), 256, 0, s>>>(n_rem, flag, cand, n, n_new,
                                                                 st.x, st.du, gt);
  if (hipGetLastError() != hipSuccess) return OTM_ERR_HIP;
  st.n_nodes = n_new;
  *inserted = k_ins;
  return OTM_OK;
}

otm_status launch_erode(otm_state& st, const otm_params& p, const Workspace& w, hipStream_t s,
                        int64_t* inserted) {
  *inserted = 0;
  const int64_t n = st.n_mp;
  if (n == 0) return OTM_OK;
  const unsigned nb = (unsigned)((n + 255) / 256);
  k_keep_flags<<<nb, 256, 0, s>>>(n, st.failed, w.mp_cell);
  scan_inclusive(w.mp_cell, n, w.scan_aux, s);
  int32_t n_keep = 0;
  if (hipMemcpyAsync(&n_keep, w.mp_cell + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return OTM_ERR_HIP;
  if (n_keep == n) return OTM_OK;
  if (p.insert_dist > 0.0 && st.n_nodes > 0) {
    const otm_status ei = insert_nodes(st, p, n - n_keep, w, inserted, s);
    if (ei != OTM_OK) return ei;
  }
  const int32_t* f = st.failed;
  otm_status e = OTM_OK;
  auto run = [&](otm_status r) { if (e == OTM_OK) e = r; };
  run(compact_field(st.xp, 3, n, n_keep, f, w, s));
  run(compact_field(st.vol, 1, n, n_keep, f, w, s));
  run(compact_field(const_cast<double*>(st.mass), 1, n, n_keep, f, w, s));  // constant but for this compaction
  run(compact_field(st.lam, 3, n, n_keep, f, w, s));
  run(compact_field(st.epsbar, 1, n, n_keep, f, w, s));
  run(compact_field(st.T, 1, n, n_keep, f, w, s));
  if (st.qflux != nullptr) run(compact_field(st.qflux, 3, n, n_keep, f, w, s));
  if (st.precision == OTM_FP64) {
    run(compact_field((double*)st.Fd, 9, n, n_keep, f, w, s));
    run(compact_field((double*)st.bed, 6, n, n_keep, f, w, s));
    run(compact_field((double*)st.sigma, 6, n, n_keep, f, w, s));
  } else {
    run(compact_field((float*)st.Fd, 9, n, n_keep, f, w, s));
    run(compact_field((float*)st.bed, 6, n, n_keep, f, w, s));
    run(compact_field((float*)st.sigma, 6, n, n_keep, f, w, s));
  }
  if (e != OTM_OK) return e;
  // the mask is read by every compaction above; the survivors' flags are 0
  if (n_keep > 0) launch_fill_i32(st.failed, n_keep, 0, s);
  if (hipGetLastError() != hipSuccess) return OTM_ERR_HIP;
  st.n_mp = n_keep;
  return OTM_OK;
}

// ------------------------------------------------ nodes in no support
__global__ void k_node_flags_clear(int64_t n, int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = 0;
}

// Every node that some pair uses is kept (all writers store the same 1).
__global__ void k_node_flags_mark(int64_t P, const int32_t* __restrict__ idx,
                                  int32_t* __restrict__ flag) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P) flag[idx[q]] = 1;
}

// Node ids of the pairs after the deletion: the kept node's rank.
__global__ void k_renumber(int64_t P, const int32_t* __restrict__ node_scan,
                           int32_t* __restrict__ idx) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P) idx[q] = node_scan[idx[q]] - 1;
}

// [ncomp][n] -> [ncomp][n_keep] for the items kept by an inclusive scan of
// keep flags (item i kept when scan[i] > scan[i - 1]).
__global__ void k_compact_by_scan(const double* __restrict__ src, double* __restrict__ dst,
                                  int64_t n, int64_t n_keep, int ncomp,
                                  const int32_t* __restrict__ scan) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t before = i > 0 ? scan[i - 1] : 0;
  if (scan[i] == before) return;
  for (int c = 0; c < ncomp; ++c) dst[c * n_keep + before] = src[c * n + i];
}

static otm_status compact_nodes(double* a, int ncomp, int64_t n, int64_t n_keep,
                                const int32_t* scan, double* tmp, hipStream_t s) {
  k_compact_by_scan<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, tmp, n, n_keep, ncomp, scan);
  if (hipGetLastError() != hipSuccess) return OTM_ERR_HIP;
  if (n_keep == 0) return OTM_OK;
  return hipMemcpyAsync(a, tmp, sizeof(double) * (size_t)ncomp * (size_t)n_keep,
                        hipMemcpyDeviceToDevice, s) == hipSuccess ? OTM_OK : OTM_ERR_HIP;
}

otm_status launch_delete_orphans(otm_state& st, const otm_params& p, const Workspace& w,
                                 hipStream_t s, int64_t* deleted) {
  *deleted = 0;
  const int64_t n = st.n_nodes;
  if (n == 0) return OTM_OK;
  int64_t P = 0;
  if (hipMemcpyAsync(&P, st.nbr_offsets + st.n_mp, sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return OTM_ERR_HIP;
  if (P > st.pair_capacity) return OTM_ERR_CAPACITY;  // the refresh's lists did not fit
  int32_t* flag = w.node_cell;
  k_node_flags_clear<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, flag);
  if (P > 0) k_node_flags_mark<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(P, st.nbr_idx, flag);
  scan_inclusive(flag, n, w.scan_aux, s);
  int32_t n_keep = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&n_keep, flag + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return OTM_ERR_HIP;
  if (n_keep == n) return OTM_OK;
  if ((size_t)3 * (size_t)n * sizeof(double) > (size_t)st.pair_capacity * sizeof(double4))
    return OTM_ERR_ARG;
  if (P > 0) k_renumber<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(P, flag, st.nbr_idx);
  double* tmp = reinterpret_cast<double*>(w.contrib);
  otm_status e = OTM_OK;
  auto run = [&](otm_status r) { if (e == OTM_OK) e = r; };
  run(compact_nodes(st.x, 3, n, n_keep, flag, tmp, s));
  run(compact_nodes(st.du, 3, n, n_keep, flag, tmp, s));
  run(compact_nodes(st.m, 1, n, n_keep, flag, tmp, s));
  run(compact_nodes(st.f, 3, n, n_keep, flag, tmp, s));
  if (p.tool_enabled) run(compact_nodes(st.tool_gt, 3, n, n_keep, flag, tmp, s));
  if (p.kappa > 0.0) run(compact_nodes(st.heat, 2, n, n_keep, flag, tmp, s));
  if (e != OTM_OK) return e;
  st.n_nodes = n_keep;
  *deleted = n - n_keep;
  return OTM_OK;
}

}  // namespace otm
