// Removal of failed material points from the body: a stable stream
// compaction of every per-MP array of the state, for otm_erode.
#include <hip/hip_runtime.h>

#include "erode.h"

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

otm_status launch_erode(otm_state& st, const Workspace& w, hipStream_t s) {
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
  const int32_t* f = st.failed;
  otm_status e = OTM_OK;
  auto run = [&](otm_status r) { if (e == OTM_OK) e = r; };
  run(compact_field(st.xp, 3, n, n_keep, f, w, s));
  run(compact_field(st.vol, 1, n, n_keep, f, w, s));
  run(compact_field(const_cast<double*>(st.mass), 1, n, n_keep, f, w, s));  // constant but for this compaction
  run(compact_field(st.lam, 3, n, n_keep, f, w, s));
  run(compact_field(st.epsbar, 1, n, n_keep, f, w, s));
  run(compact_field(st.T, 1, n, n_keep, f, w, s));
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

}  // namespace otm
