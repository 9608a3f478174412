// Support-domain search with linked cells (Sec. 3, Alg. 3), plus the prefix
// sums and small fills the library needs.
//
// Nodes are binned into static cells of edge >= r_list over their bounding
// box; a copy of the node coordinates is stored in cell order (x, y, z, id
// as one 32-byte record) so the 27-cell scan of an MP reads contiguous
// memory.  Each MP's nodes are kept sorted by id in LDS while they are found,
// so lists come out in canonical order.  The squared distance is evaluated as
// ((dx*dx + dy*dy) + dz*dz) with every operation rounded separately.
#include "launch.h"
#include "otm_common.h"

namespace otm {

// ---------------------------------------------------------------- prefix sum
template <typename T>
__global__ __launch_bounds__(1024) void k_scan_blocks(T* a, int64_t n, int64_t* aux) {
  __shared__ T s[1024];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * 4;
  T v[4];
  T run = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k;
    run += (i < n) ? a[i] : T(0);
    v[k] = run;
  }
  s[tid] = run;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const T add = tid >= o ? s[tid - o] : T(0);
    __syncthreads();
    s[tid] += add;
    __syncthreads();
  }
  const T excl = tid > 0 ? s[tid - 1] : T(0);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k;
    if (i < n) a[i] = v[k] + excl;
  }
  if (tid == 1023) aux[blockIdx.x] = (int64_t)s[1023];
}

// Exclusive scan of the block totals by one workgroup (any count).
__global__ __launch_bounds__(1024) void k_scan_aux(int64_t* aux, int64_t nb) {
  __shared__ int64_t s[1024];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    const int64_t i = b0 + tid;
    const int64_t v = i < nb ? aux[i] : 0;
    s[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int64_t add = tid >= o ? s[tid - o] : 0;
      __syncthreads();
      s[tid] += add;
      __syncthreads();
    }
    if (i < nb) aux[i] = carry + s[tid] - v;
    __syncthreads();
    if (tid == 0) carry += s[1023];
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_add(T* a, int64_t n, const int64_t* aux) {
  const int64_t add = aux[blockIdx.x];
  if (add == 0) return;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  for (int k = threadIdx.x; k < kScanBlock; k += 1024) {
    const int64_t i = base + k;
    if (i < n) a[i] += (T)add;
  }
}

template <typename T>
static void scan_impl(T* a, int64_t n, int64_t* aux, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  k_scan_blocks<T><<<dim3((unsigned)nb), dim3(1024), 0, s>>>(a, n, aux);
  if (nb > 1) {
    k_scan_aux<<<1, 1024, 0, s>>>(aux, nb);
    k_scan_add<T><<<dim3((unsigned)nb), dim3(1024), 0, s>>>(a, n, aux);
  }
}
void scan_inclusive(int64_t* a, int64_t n, int64_t* aux, hipStream_t s) { scan_impl(a, n, aux, s); }
void scan_inclusive(int32_t* a, int64_t n, int64_t* aux, hipStream_t s) { scan_impl(a, n, aux, s); }

// ---------------------------------------------------------------- fills
__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
__global__ void k_fill_f64(double* a, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
static unsigned fill_blocks(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}
void launch_zero(double* a, int64_t n, hipStream_t s) {
  if (n > 0) k_fill_f64<<<fill_blocks(n), 256, 0, s>>>(a, n, 0.0);
}
__global__ void k_fill_i64(int64_t* a, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t s) {
  if (n > 0) k_fill_i32<<<fill_blocks(n), 256, 0, s>>>(a, n, v);
}
void launch_fill_i64(int64_t* a, int64_t n, int64_t v, hipStream_t s) {
  if (n > 0) k_fill_i64<<<fill_blocks(n), 256, 0, s>>>(a, n, v);
}
static void fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t s) { launch_fill_i32(a, n, v, s); }

__global__ void k_diag_reset(otm_diag* d) {
  d->flags = 0;
  d->max_support = 0;
  d->n_lme_noconv = d->n_rm_noconv = d->n_inverted = d->n_nonfinite = 0;
  d->first_lme_noconv = d->first_rm_noconv = d->first_inverted = d->first_nonfinite = ~0ull;
  d->pairs_needed = 0;
  d->reserved[0] = d->reserved[1] = d->reserved[2] = 0;
}
void launch_diag_reset(otm_diag* d, hipStream_t s) { k_diag_reset<<<1, 1, 0, s>>>(d); }

// ---------------------------------------------------------------- cell grid
__global__ __launch_bounds__(256) void k_bbox_partial(const double* x, int64_t n, double* part) {
  __shared__ double sh[6][256];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = x[c * n + i];
      lo[c] = fmin(lo[c], v);
      hi[c] = fmax(hi[c], v);
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) { sh[c][threadIdx.x] = lo[c]; sh[3 + c][threadIdx.x] = hi[c]; }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + o]);
        sh[3 + c][threadIdx.x] = fmax(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + o]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 6; ++c) part[blockIdx.x * 6 + c] = sh[c][0];
}

// Grid over the box: cell edge = cell_size, enlarged by 1.25x until the cell
// count fits the workspace (a larger cell only adds candidates).  Non-finite
// extents fall back to a single cell of unbounded size; every coordinate is
// clamped into the grid, so no cell index can leave it.
__global__ __launch_bounds__(256) void k_grid_finalize(const double* part, int nb,
                                                       double cell_size, int64_t cap, Grid* g) {
  __shared__ double sh[6][256];
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += 256)
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], part[b * 6 + c]);
      hi[c] = fmax(hi[c], part[b * 6 + 3 + c]);
    }
  for (int c = 0; c < 3; ++c) { sh[c][threadIdx.x] = lo[c]; sh[3 + c][threadIdx.x] = hi[c]; }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int c = 0; c < 3; ++c) {
        sh[c][threadIdx.x] = fmin(sh[c][threadIdx.x], sh[c][threadIdx.x + o]);
        sh[3 + c][threadIdx.x] = fmax(sh[3 + c][threadIdx.x], sh[3 + c][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  for (int c = 0; c < 3; ++c) { lo[c] = sh[c][0]; hi[c] = sh[3 + c][0]; }
  double ext[3];
  bool finite = true;
  for (int c = 0; c < 3; ++c) {
    ext[c] = hi[c] - lo[c];
    if (!isfinite(ext[c]) || !isfinite(lo[c])) finite = false;
    if (!(ext[c] > 0.0)) ext[c] = 0.0;
  }
  double cell = cell_size;
  int64_t dims[3] = {1, 1, 1}, total = 1;
  bool fits = false;
  for (int tries = 0; finite && tries < 400; ++tries) {
    double dd[3], tot = 1.0;
    for (int c = 0; c < 3; ++c) {
      dd[c] = floor(ext[c] / cell) + 1.0;
      tot *= dd[c];
    }
    if (tot <= (double)cap) {
      total = 1;
      for (int c = 0; c < 3; ++c) {
        dims[c] = (int64_t)dd[c];
        total *= dims[c];
      }
      fits = true;
      break;
    }
    cell *= 1.25;
  }
  if (!fits) {
    dims[0] = dims[1] = dims[2] = 1;
    total = 1;
    cell = INFINITY;
    for (int c = 0; c < 3; ++c) lo[c] = isfinite(lo[c]) ? lo[c] : 0.0;
  }
  for (int c = 0; c < 3; ++c) { g->lo[c] = lo[c]; g->dims[c] = (int32_t)dims[c]; }
  g->cell = cell;
  g->n_cells = total;
}

OTM_DEV int cell_coord(double x, double lo, double inv_cell, int dim) {
  const double t = floor((x - lo) * inv_cell);
  // NaN lands in cell 0 (non-finite positions are reported by the MP update)
  int c = !(t >= 0.0) ? 0 : (t > (double)(dim - 1) ? dim - 1 : (int)t);
  return c;
}

__global__ void k_bin_count(const double* x, int64_t n, const Grid* g, int32_t* node_cell,
                            int32_t* cell_start) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double inv = 1.0 / g->cell;
  const int cx = cell_coord(x[i], g->lo[0], inv, g->dims[0]);
  const int cy = cell_coord(x[n + i], g->lo[1], inv, g->dims[1]);
  const int cz = cell_coord(x[2 * n + i], g->lo[2], inv, g->dims[2]);
  const int32_t cid = (cz * g->dims[1] + cy) * g->dims[0] + cx;
  node_cell[i] = cid;
  atomicAdd(&cell_start[cid + 1], 1);
}

__global__ void k_bin_fill(const double* x, int64_t n, const int32_t* node_cell,
                           const int32_t* cell_start, int32_t* cursor, double4* sorted) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t cid = node_cell[i];
  const int32_t pos = cell_start[cid] + atomicAdd(&cursor[cid], 1);
  sorted[pos] = make_double4(x[i], x[n + i], x[2 * n + i], (double)i);
}

// ---------------------------------------------------------------- MP lists
OTM_DEV double sqdist(double ax, double ay, double az, double bx, double by, double bz) {
#pragma clang fp contract(off)
  const double dx = ax - bx, dy = ay - by, dz = az - bz;
  return (dx * dx + dy * dy) + dz * dz;
}

// Visits every node within r of (px,py,pz), in cell order.
template <typename Visit>
OTM_DEV void for_each_neighbor(double px, double py, double pz, double r2, const Grid& g,
                               const int32_t* __restrict__ cell_start,
                               const double4* __restrict__ sorted, Visit&& visit) {
  const double inv = 1.0 / g.cell;
  const int cx = cell_coord(px, g.lo[0], inv, g.dims[0]);
  const int cy = cell_coord(py, g.lo[1], inv, g.dims[1]);
  const int cz = cell_coord(pz, g.lo[2], inv, g.dims[2]);
  for (int z = cz - 1; z <= cz + 1; ++z) {
    if (z < 0 || z >= g.dims[2]) continue;
    for (int y = cy - 1; y <= cy + 1; ++y) {
      if (y < 0 || y >= g.dims[1]) continue;
      const int row = (z * g.dims[1] + y) * g.dims[0];
      const int x0 = cx > 0 ? cx - 1 : 0;
      const int x1 = cx + 1 < g.dims[0] ? cx + 1 : g.dims[0] - 1;
      // cells x0..x1 of one row are contiguous in the sorted array
      const int32_t s0 = cell_start[row + x0], s1 = cell_start[row + x1 + 1];
      for (int32_t s = s0; s < s1; ++s) {
        const double4 nd = sorted[s];
        if (sqdist(px, py, pz, nd.x, nd.y, nd.z) <= r2) visit((int32_t)nd.w);
      }
    }
  }
}

// One pass over the 27 cells per MP.  A group of 8 lanes shares one MP: the
// lanes test consecutive node records of each row of cells together (so a
// load instruction touches few cache lines), hits are appended to the MP's
// list in LDS by a ballot prefix count, and the list is then put in
// ascending id order by a rank sort (ids are distinct).  The count goes to
// offsets[p+1] and the sorted row to the block's staging area, rows of
// kRowCap ids per MP, contiguous per workgroup.  Longer rows are only
// counted here and re-found by the compaction kernel.
constexpr int kScanThreads = 256;
constexpr int kScanLanes = 8;
constexpr int kScanMPs = 64;   // MPs per workgroup (two rounds of 32 groups)
constexpr int kScanUnroll = 4;
constexpr int kRowCap = kRowCapacity;

__global__ __launch_bounds__(kScanThreads) void k_nbr_scan(
    const double* __restrict__ xp, int64_t n_mp, double r2, const Grid* __restrict__ gp,
    const int32_t* __restrict__ cell_start, const double4* __restrict__ sorted,
    int64_t* __restrict__ offsets, int32_t* __restrict__ stage, int32_t* __restrict__ block_max) {
  __shared__ int32_t found[kScanThreads / kScanLanes][kRowCap];
  __shared__ int32_t red[kScanThreads];
  int32_t nmax = 0;
  const int tid = threadIdx.x, grp = tid / kScanLanes, lane = tid % kScanLanes;
  const int wave_grp = (tid % kWave) / kScanLanes;  // group index inside the wave
  const int64_t blk = xcd_block();
  if (blk == 0 && tid == 0) offsets[0] = 0;
  const Grid g = *gp;
  for (int r = 0; r < kScanMPs / (kScanThreads / kScanLanes); ++r) {
    const int local = r * (kScanThreads / kScanLanes) + grp;
    const int64_t p = blk * kScanMPs + local;
    const bool valid = p < n_mp;
    int32_t n = 0;
    if (valid) {
      const double px = xp[p], py = xp[n_mp + p], pz = xp[2 * n_mp + p];
      // the 9 row ranges, loaded together; candidates are then taken as one
      // flat list, kScanUnroll chunks of 8 per iteration with independent loads
      int32_t rs[9], pre[10];
      {
        const double inv = 1.0 / g.cell;
        const int cx = cell_coord(px, g.lo[0], inv, g.dims[0]);
        const int cy = cell_coord(py, g.lo[1], inv, g.dims[1]);
        const int cz = cell_coord(pz, g.lo[2], inv, g.dims[2]);
        const int x0 = cx > 0 ? cx - 1 : 0;
        const int x1 = cx + 1 < g.dims[0] ? cx + 1 : g.dims[0] - 1;
        int32_t re[9];
        // branch-free: every load is issued (clamped rows), then masked
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const int z = cz - 1 + k / 3, y = cy - 1 + k % 3;
          const bool in = z >= 0 && z < g.dims[2] && y >= 0 && y < g.dims[1];
          const int zc = z < 0 ? 0 : (z >= g.dims[2] ? g.dims[2] - 1 : z);
          const int yc = y < 0 ? 0 : (y >= g.dims[1] ? g.dims[1] - 1 : y);
          const int rw = (zc * g.dims[1] + yc) * g.dims[0];
          const int32_t a = cell_start[rw + x0], b = cell_start[rw + x1 + 1];
          rs[k] = in ? a : 0;
          re[k] = in ? b : 0;
        }
        pre[0] = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) pre[k + 1] = pre[k] + (re[k] - rs[k]);
      }
      const int32_t total = pre[9];
      for (int32_t b = 0; b < total; b += kScanLanes * kScanUnroll) {
        double4 nd[kScanUnroll];
        bool in[kScanUnroll];
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) {
          const int32_t c = b + u * kScanLanes + lane;
          in[u] = c < total;
          int32_t shift = rs[0] - pre[0];
#pragma unroll
          for (int k = 1; k < 9; ++k) shift = c >= pre[k] ? rs[k] - pre[k] : shift;
          nd[u] = sorted[in[u] ? c + shift : 0];  // record 0 stands in past the end
        }
#pragma unroll
        for (int u = 0; u < kScanUnroll; ++u) {
          const bool hit = in[u] && sqdist(px, py, pz, nd[u].x, nd[u].y, nd[u].z) <= r2;
          const uint64_t m = __ballot(hit);
          const uint32_t gm = (uint32_t)(m >> (wave_grp * kScanLanes)) & 0xffu;
          const int pos = n + __popc(gm & ((1u << lane) - 1u));
          if (hit && pos < kRowCap) found[grp][pos] = (int32_t)nd[u].w;
          n += __popc(gm);
        }
      }
    }
    // the group's lanes read each other's LDS writes below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (valid) {
      if (lane == 0) offsets[p + 1] = n;
      nmax = n > nmax ? n : nmax;
      if (n <= kRowCap) {
        int32_t* row = stage + (blk * kScanMPs + local) * kRowCap;
        for (int e = lane; e < n; e += kScanLanes) {
          const int32_t v = found[grp][e];
          int rank = 0;
          for (int j = 0; j < n; ++j) rank += found[grp][j] < v;
          row[rank] = v;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // largest support of the workgroup (reduced once more by k_search_done;
  // one atomic per MP on a single counter would serialise the whole pass)
  red[tid] = nmax;
  __syncthreads();
  for (int o = kScanThreads / 2; o > 0; o >>= 1) {
    if (tid < o) red[tid] = red[tid] > red[tid + o] ? red[tid] : red[tid + o];
    __syncthreads();
  }
  if (tid == 0) block_max[blk] = red[0];
}

// Copies each workgroup's staged rows into its contiguous CSR segment with
// unit-stride stores; rows longer than kRowCap are found again and sorted
// in place by their own lane.
__global__ __launch_bounds__(256) void k_nbr_compact(
    const double* __restrict__ xp, int64_t n_mp, double r2, const Grid* __restrict__ gp,
    const int32_t* __restrict__ cell_start, const double4* __restrict__ sorted,
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ stage, int64_t capacity,
    int32_t* __restrict__ idx) {
  __shared__ int32_t rows[kScanMPs * kRowCap];
  __shared__ int64_t off[kScanMPs + 1];
  const int tid = threadIdx.x;
  const int64_t blk = xcd_block();
  const int64_t p0 = blk * kScanMPs;
  if (p0 >= n_mp) return;
  if (offsets[n_mp] > capacity) return;  // lists do not fit: counts only
  const int nloc = (int)(n_mp - p0 < kScanMPs ? n_mp - p0 : kScanMPs);
  for (int i = tid; i <= nloc; i += 256) off[i] = offsets[p0 + i];
  for (int i = tid; i < nloc * kRowCap; i += 256) rows[i] = stage[p0 * kRowCap + i];
  __syncthreads();
  const int64_t base = off[0];
  const int total = (int)(off[nloc] - base);
  for (int e = tid; e < total; e += 256) {
    // MP of output element e: last t with off[t] - base <= e
    int lo = 0, hi = nloc - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] - base <= e) lo = mid; else hi = mid - 1;
    }
    const int K = (int)(off[lo + 1] - off[lo]);
    if (K <= kRowCap) idx[base + e] = rows[lo * kRowCap + (e - (int)(off[lo] - base))];
  }
  // long supports
  if (tid < nloc && off[tid + 1] - off[tid] > kRowCap) {
    const int64_t p = p0 + tid;
    const int64_t o = off[tid];
    const Grid g = *gp;
    int32_t n = 0;
    for_each_neighbor(xp[p], xp[n_mp + p], xp[2 * n_mp + p], r2, g, cell_start, sorted,
                      [&](int32_t id) {
                        int32_t j = n++;
                        while (j > 0 && idx[o + j - 1] > id) {
                          idx[o + j] = idx[o + j - 1];
                          --j;
                        }
                        idx[o + j] = id;
                      });
  }
}

__global__ void k_set_first_offset(int64_t* offsets) { offsets[0] = 0; }

__global__ __launch_bounds__(256) void k_search_done(const int64_t* offsets, int64_t n_mp,
                                                     const int32_t* block_max, int64_t nblocks,
                                                     int64_t capacity, otm_diag* diag) {
  __shared__ int32_t red[256];
  int32_t m = 0;
  for (int64_t b = threadIdx.x; b < nblocks; b += 256) m = block_max[b] > m ? block_max[b] : m;
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + o] ? red[threadIdx.x]
                                                                 : red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x != 0 || diag == nullptr) return;
  const int64_t P = offsets[n_mp];
  diag->pairs_needed = P;
  diag->max_support = red[0];
  if (P > capacity) atomicOr(&diag->flags, 1u << (-OTM_ERR_CAPACITY - 1));
}

void launch_search(int64_t n_nodes, const double* x_nodes, int64_t n_mp, const double* x_mp,
                   double r_list, double cell_size, int64_t pair_capacity, int64_t* nbr_offsets,
                   int32_t* nbr_idx, const Workspace& w, otm_diag* diag, hipStream_t s) {
  k_bbox_partial<<<kBBoxBlocks, 256, 0, s>>>(x_nodes, n_nodes, w.bbox_part);
  k_grid_finalize<<<1, 256, 0, s>>>(w.bbox_part, kBBoxBlocks, cell_size, w.cap_cells, w.grid);
  fill_i32(w.cell_start, w.cap_cells + 1, 0, s);
  fill_i32(w.cell_cursor, w.cap_cells, 0, s);
  const unsigned nbn = (unsigned)((n_nodes + 255) / 256);
  if (nbn > 0)
    k_bin_count<<<nbn, 256, 0, s>>>(x_nodes, n_nodes, w.grid, w.node_cell, w.cell_start);
  scan_inclusive(w.cell_start + 1, w.cap_cells, w.scan_aux, s);
  if (nbn > 0)
    k_bin_fill<<<nbn, 256, 0, s>>>(x_nodes, n_nodes, w.node_cell, w.cell_start, w.cell_cursor,
                                   w.sorted);
  const double r2 = r_list * r_list;
  if (n_mp > 0) {
    const unsigned nbs = (unsigned)((n_mp + kScanMPs - 1) / kScanMPs);
    k_nbr_scan<<<nbs, kScanThreads, 0, s>>>(x_mp, n_mp, r2, w.grid, w.cell_start, w.sorted,
                                            nbr_offsets, w.stage, w.block_max);
    scan_inclusive(nbr_offsets + 1, n_mp, w.scan_aux, s);
    k_nbr_compact<<<nbs, 256, 0, s>>>(
        x_mp, n_mp, r2, w.grid, w.cell_start, w.sorted, nbr_offsets, w.stage, pair_capacity,
        nbr_idx);
  } else {
    k_set_first_offset<<<1, 1, 0, s>>>(nbr_offsets);
  }
  const int64_t nbs_all = (n_mp + kScanMPs - 1) / kScanMPs;
  k_search_done<<<1, 256, 0, s>>>(nbr_offsets, n_mp, w.block_max, nbs_all, pair_capacity, diag);
}

}  // namespace otm
