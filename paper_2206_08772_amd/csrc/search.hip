// Support-domain search with linked cells (Sec. 3, Alg. 3), plus the prefix
// sums and small fills the library needs.
//
// Nodes are binned into static cells of edge >= r_list over their bounding
// box; a copy of the node coordinates is stored in cell order (x, y, z, id
// as one 32-byte record) so the 27-cell scan of an MP reads contiguous
// memory.  Each MP's nodes are kept sorted by id in LDS while they are found,
// so lists come out in canonical order.  The squared distance is evaluated as
// ((dx*dx + dy*dy) + dz*dz) with every operation rounded separately.
#include <type_traits>

#include "launch.h"
#include "otm_common.h"

namespace otm {

// ---------------------------------------------------------------- prefix sum
// Inclusive scan in three passes: each workgroup scans kScanBlock elements
// and writes its total, one workgroup scans the totals (exclusive), each
// workgroup adds its offset.  Two arrays of equal length (the node and MP
// cell counts) go through the same three launches: workgroup b works on
// array b / nb, and the totals of each array are scanned separately.
template <typename T>
OTM_DEV void scan_block(T* a, int64_t n, int64_t blk, int64_t* total) {
  __shared__ T s[1024];
  const int tid = threadIdx.x;
  const int64_t base = blk * kScanBlock + (int64_t)tid * 4;
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
  if (tid == 1023) *total = (int64_t)s[1023];
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_blocks(T* a, T* b, int64_t n, int64_t nb,
                                                      int64_t* aux) {
  const int64_t seg = blockIdx.x / nb;
  scan_block(seg == 0 ? a : b, n, blockIdx.x - seg * nb, aux + blockIdx.x);
}

// Exclusive scan of nseg segments of nb block totals by one workgroup.
__global__ __launch_bounds__(1024) void k_scan_aux(int64_t* aux, int64_t nb, int nseg) {
  __shared__ int64_t s[1024];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  for (int seg = 0; seg < nseg; ++seg) {
    int64_t* t = aux + seg * nb;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
      const int64_t i = b0 + tid;
      const int64_t v = i < nb ? t[i] : 0;
      s[tid] = v;
      __syncthreads();
      for (int o = 1; o < 1024; o <<= 1) {
        const int64_t add = tid >= o ? s[tid - o] : 0;
        __syncthreads();
        s[tid] += add;
        __syncthreads();
      }
      if (i < nb) t[i] = carry + s[tid] - v;
      __syncthreads();
      if (tid == 0) carry += s[1023];
      __syncthreads();
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_add(T* a, T* b, int64_t n, int64_t nb,
                                                   const int64_t* aux) {
  const int64_t add = aux[blockIdx.x];
  if (add == 0) return;
  const int64_t seg = blockIdx.x / nb;
  T* arr = seg == 0 ? a : b;
  const int64_t base = (blockIdx.x - seg * nb) * kScanBlock;
  for (int k = threadIdx.x; k < kScanBlock; k += 1024) {
    const int64_t i = base + k;
    if (i < n) arr[i] += (T)add;
  }
}

// b == nullptr: one array
template <typename T>
static void scan_impl(T* a, T* b, int64_t n, int64_t* aux, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  const int nseg = b == nullptr ? 1 : 2;
  const unsigned grid = (unsigned)(nb * nseg);
  k_scan_blocks<T><<<grid, 1024, 0, s>>>(a, b, n, nb, aux);
  if (nb > 1) {
    k_scan_aux<<<1, 1024, 0, s>>>(aux, nb, nseg);
    k_scan_add<T><<<grid, 1024, 0, s>>>(a, b, n, nb, aux);
  }
}
void scan_inclusive(int64_t* a, int64_t n, int64_t* aux, hipStream_t s) {
  scan_impl<int64_t>(a, nullptr, n, aux, s);
}
void scan_inclusive(int32_t* a, int64_t n, int64_t* aux, hipStream_t s) {
  scan_impl<int32_t>(a, nullptr, n, aux, s);
}

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
// Bounding box partials of the nodes; the same launch clears the cell
// counters and cursors of the node and MP binnings that follow.
struct BinCounters {
  int32_t* node_start;  // [cap + 1]
  int32_t* node_cursor; // [cap]
  int32_t* mp_start;    // [cap + 1]
  int32_t* mp_cursor;   // [cap]
  int64_t cap;
};

__global__ __launch_bounds__(256) void k_bbox_partial(const double* x, int64_t n, double* part,
                                                      BinCounters z) {
  __shared__ double sh[6][256];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= z.cap;
       i += (int64_t)gridDim.x * blockDim.x) {
    z.node_start[i] = 0;
    z.mp_start[i] = 0;
    if (i < z.cap) {
      z.node_cursor[i] = 0;
      z.mp_cursor[i] = 0;
    }
  }
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

// Counting sort of two point sets (nodes, then MPs) on one grid, each pass
// one launch: thread i < n_a takes point i of set a, threads from b0 (n_a
// rounded up to a wave, so no wave mixes the sets and the wave-grouped
// atomics see one counter array) take set b.
struct BinSet {
  const double* x;     // [3][n]
  int64_t n;
  int32_t* cell;       // [n] cell of each point
  int32_t* start;      // [cap + 1] counts, then offsets
  int32_t* cursor;     // [cap]
  double4* sorted;     // [n] (x, y, z, index) in cell order
};

OTM_DEV bool bin_pick(const BinSet& a, const BinSet& b, int64_t b0, const BinSet*& set,
                      int64_t& i) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < a.n) { set = &a; i = t; return true; }
  if (t >= b0 && t - b0 < b.n) { set = &b; i = t - b0; return true; }
  return false;
}

__global__ __launch_bounds__(256) void k_bin_count(BinSet a, BinSet b, int64_t b0,
                                                   const Grid* g) {
  const BinSet* set;
  int64_t i;
  if (!bin_pick(a, b, b0, set, i)) return;
  const double* x = set->x;
  const int64_t n = set->n;
  const double inv = 1.0 / g->cell;
  const int cx = cell_coord(x[i], g->lo[0], inv, g->dims[0]);
  const int cy = cell_coord(x[n + i], g->lo[1], inv, g->dims[1]);
  const int cz = cell_coord(x[2 * n + i], g->lo[2], inv, g->dims[2]);
  const int32_t cid = (cz * g->dims[1] + cy) * g->dims[0] + cx;
  set->cell[i] = cid;
  grouped_atomic_add(set->start + 1, cid);
}

__global__ __launch_bounds__(256) void k_bin_fill(BinSet a, BinSet b, int64_t b0) {
  const BinSet* set;
  int64_t i;
  if (!bin_pick(a, b, b0, set, i)) return;
  const double* x = set->x;
  const int64_t n = set->n;
  const int32_t cid = set->cell[i];
  const int32_t pos = set->start[cid] + grouped_atomic_add(set->cursor, cid);
  set->sorted[pos] = make_double4(x[i], x[n + i], x[2 * n + i], (double)i);
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

// Row ranges of the 27 cells around cell (cx, cy, cz): the 9 (z, y) rows of
// three cells each are contiguous in the binned array.  Rows outside the
// grid are empty.  pre[k] is the number of candidates before row k.
OTM_DEV void cell_rows(const Grid& g, const int32_t* __restrict__ cell_start, int cx, int cy,
                       int cz, int32_t rs[9], int32_t pre[10]) {
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

// Position in the binned array of candidate c (0 <= c < pre[9]).
OTM_DEV int32_t cand_pos(int32_t c, const int32_t rs[9], const int32_t pre[10]) {
  int32_t shift = rs[0] - pre[0];
#pragma unroll
  for (int k = 1; k < 9; ++k) shift = c >= pre[k] ? rs[k] - pre[k] : shift;
  return c + shift;
}

OTM_DEV void wave_sync() {
  // the wave's lanes read each other's LDS writes after this point
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

OTM_DEV double lane_value(double v, int t) {  // v of lane t (t uniform)
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, t);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), t);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Cell-centric pass: one wave per grid cell.  All MPs of a cell have the same
// 27 candidate cells, so the wave loads the candidates once and keeps them in
// registers, lane l holding candidates l, l + 64, ...  Each MP of the cell
// (binned like the nodes) is then tested against them: a ballot of the hits,
// taken in candidate order, gives each hit its place in the MP's staging
// row.  The row is in stencil order; the compaction sorts it by node id (the
// four lanes of a quad per row, in registers), which costs far fewer
// instructions than sorting each cell's candidates.  The count goes to offsets[p + 1]; rows
// longer than kRowCap are only counted (the compaction re-finds them).  A
// cell with more than kCand candidates takes each MP separately: hits are
// appended to LDS by ballot and rank-sorted.
//
// The cell index is wave-uniform, so a cell's header (MP range, candidate
// rows) comes from scalar loads, and the next cell's header is requested
// before the current cell is processed.  Each XCD strides over its own
// contiguous eighth of the cells (neighbouring cells share that XCD's L2).
constexpr int kCellWaves = 4;
constexpr unsigned kCellBlocks = 8 * 1024;
constexpr int kCand = 320;
constexpr int kCandChunks = kCand / kWave;
constexpr int kRowCap = kRowCapacity;

struct CellHdr {
  int32_t m0, m1;
  int32_t rs[9], pre[10];
};

OTM_DEV CellHdr cell_header(int64_t c, const Grid& g, const int32_t* __restrict__ cell_start,
                            const int32_t* __restrict__ mp_cell_start) {
  CellHdr h;
  h.m0 = mp_cell_start[c];
  h.m1 = mp_cell_start[c + 1];
  const int32_t ci = (int32_t)c;  // cell counts stay below 2^31
  const int cx = ci % g.dims[0];
  const int cy = (ci / g.dims[0]) % g.dims[1];
  const int cz = ci / (g.dims[0] * g.dims[1]);
  cell_rows(g, cell_start, cx, cy, cz, h.rs, h.pre);
  return h;
}

struct CellLds {  // the hits of one MP in the dense path
  int32_t ids[kCand];
};

OTM_DEV void cell_scan_one(const CellHdr& h, double r2, const double4* __restrict__ sorted,
                           const double4* __restrict__ mp_sorted, int64_t* __restrict__ offsets,
                           int32_t* __restrict__ stage, CellLds& L, int lane) {
  const int32_t m0 = h.m0, m1 = h.m1;
  if (m0 == m1) return;
  const int32_t T = h.pre[9];
  if (T <= kCand) {
    const int nch = (T + kWave - 1) / kWave;  // uniform
    double4 v[kCandChunks];
    // the first 64 MPs of the cell, requested with the candidates
    const int mc0 = m1 - m0 < kWave ? (int)(m1 - m0) : kWave;
    double4 mine = mp_sorted[m0 + (lane < mc0 ? lane : mc0 - 1)];
    // the candidates in stencil order: the rows come out unsorted and the
    // compaction sorts each one by node id
#pragma unroll
    for (int k = 0; k < kCandChunks; ++k) {
      if (k < nch) {
        const int32_t j = k * kWave + lane;
        v[k] = sorted[cand_pos(j < T ? j : 0, h.rs, h.pre)];
      }
    }
    // per chunk: lanes holding a real candidate, and the candidate ids
    bool valid[kCandChunks];
    int32_t cid[kCandChunks];
#pragma unroll
    for (int k = 0; k < kCandChunks; ++k) {
      valid[k] = k * kWave + lane < T;
      cid[k] = (int32_t)v[k].w;
    }
    // NM MPs of the cell (lanes t .. t + NM - 1 of ``mine``) tested together:
    // their chains are independent, so the hardware overlaps them
    auto test_mps = [&](auto nm_tag, int t, int32_t pl) {
      constexpr int NM = decltype(nm_tag)::value;
      double px[NM], py[NM], pz[NM];
      int32_t* row[NM];
      int32_t p[NM];
      uint32_t n[NM];
#pragma unroll
      for (int i = 0; i < NM; ++i) {
        px[i] = lane_value(mine.x, t + i);
        py[i] = lane_value(mine.y, t + i);
        pz[i] = lane_value(mine.z, t + i);
        p[i] = __builtin_amdgcn_readlane(pl, t + i);
        row[i] = stage + (int64_t)p[i] * kRowCap;
        n[i] = 0;
      }
#pragma unroll
      for (int k = 0; k < kCandChunks; ++k) {
        if (k < nch) {
#pragma unroll
          for (int i = 0; i < NM; ++i) {
            // every lane computes the distance (stand-ins are masked), so no
            // branch around it
            const bool hit = (sqdist(px[i], py[i], pz[i], v[k].x, v[k].y, v[k].z) <= r2) &
                             valid[k];
            const uint64_t m = __ballot(hit);
            const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, n[i]));
            if (hit & (pos < (uint32_t)kRowCap)) row[i][pos] = cid[k];
            n[i] += (uint32_t)__popcll(m);
          }
        }
      }
      if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NM; ++i) offsets[p[i] + 1] = n[i];
      }
    };
    for (int32_t mb = m0; mb < m1; mb += kWave) {
      const int mc = m1 - mb < kWave ? (int)(m1 - mb) : kWave;
      if (mb != m0) mine = mp_sorted[mb + (lane < mc ? lane : mc - 1)];
      const int32_t pl = (int32_t)mine.w;  // this lane's MP
      int t = 0;
      for (; t + 3 < mc; t += 4) test_mps(std::integral_constant<int, 4>{}, t, pl);
      if (t + 1 < mc) { test_mps(std::integral_constant<int, 2>{}, t, pl); t += 2; }
      if (t < mc) test_mps(std::integral_constant<int, 1>{}, t, pl);
    }
  } else {
    // dense neighbourhood: one MP at a time, candidates read from memory
    for (int32_t m = m0; m < m1; ++m) {
      const double4 mp = mp_sorted[m];
      const int64_t p = (int64_t)mp.w;
      int32_t n = 0;
      for (int32_t b = 0; b < T; b += kWave) {
        const int32_t j = b + lane;
        const double4 nd = sorted[cand_pos(j < T ? j : 0, h.rs, h.pre)];
        const bool hit = j < T && sqdist(mp.x, mp.y, mp.z, nd.x, nd.y, nd.z) <= r2;
        const uint64_t msk = __ballot(hit);
        const int pos = n + (int)__builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(msk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)msk, 0u));
        if (hit && pos < kCand) L.ids[pos] = (int32_t)nd.w;
        n += __popcll(msk);
      }
      wave_sync();
      if (n <= kRowCap) {
        int32_t* row = stage + p * kRowCap;
        if (lane < n) {
          const int32_t id = L.ids[lane];
          int rk = 0;
          for (int t = 0; t < n; ++t) rk += L.ids[t] < id;
          row[rk] = id;
        }
      }
      if (lane == 0) offsets[p + 1] = n;
      wave_sync();
    }
  }
}

__global__ __launch_bounds__(kCellWaves * kWave) void k_cell_scan(
    double r2, const Grid* __restrict__ gp, int64_t cap_cells,
    const int32_t* __restrict__ cell_start, const double4* __restrict__ sorted,
    const int32_t* __restrict__ mp_cell_start, const double4* __restrict__ mp_sorted,
    int64_t* __restrict__ offsets, int32_t* __restrict__ stage) {
  __shared__ CellLds lds[kCellWaves];
  // wave index as a uniform value, so the cell loop runs on scalar registers
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int lane = (int)(threadIdx.x % kWave);
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[0] = 0;
  const Grid g = *gp;
  const int64_t n_cells = g.n_cells < cap_cells ? g.n_cells : cap_cells;
  const int64_t per_xcd = (n_cells + 7) / 8;
  const int64_t c_lo = (int64_t)(blockIdx.x % 8u) * per_xcd;
  const int64_t c_hi = c_lo + per_xcd < n_cells ? c_lo + per_xcd : n_cells;
  const int64_t stride = (int64_t)(gridDim.x / 8u) * kCellWaves;
  int64_t c = c_lo + (int64_t)(blockIdx.x / 8u) * kCellWaves + w;
  if (c >= c_hi) return;
  CellHdr h = cell_header(c, g, cell_start, mp_cell_start);
  for (; c < c_hi; c += stride) {
    const int64_t cn = c + stride < c_hi ? c + stride : c;
    const CellHdr hn = cell_header(cn, g, cell_start, mp_cell_start);  // next cell, early
    cell_scan_one(h, r2, sorted, mp_sorted, offsets, stage, lds[w], lane);
    h = hn;
  }
}

constexpr int kScanMPs = 64;  // MPs per compaction workgroup

// Ascending order of a staged row of K <= 32 node ids (distinct), sorted by
// the four lanes of a quad: a bitonic network over 32 slots (the slots past
// K padded with INT32_MAX), lane l of the quad holding slots 8l .. 8l + 7.
// Compare-exchanges between slots 8 or 16 apart pair a lane with the quad
// lane l ^ 1 or l ^ 2 (DPP quad permutations); the others stay in the lane.
// Every lane of the quad must call it with the same row.
OTM_DEV void sort_row32_quad(int32_t* row, int K, int l) {
  int32_t a[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) a[e] = 8 * l + e < K ? row[8 * l + e] : INT32_MAX;
#pragma unroll
  for (int k = 2; k <= 32; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 8) {
        const bool lower = (l & (j >> 3)) == 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int32_t w = j == 8 ? dpp_move<0xB1>(a[e]) : dpp_move<0x4E>(a[e]);
          const int32_t lo = a[e] < w ? a[e] : w, hi = a[e] < w ? w : a[e];
          const bool up = ((8 * l + e) & k) == 0;
          a[e] = lower == up ? lo : hi;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int f = e ^ j;
          if (f > e) {
            const int32_t x = a[e], y = a[f];
            const int32_t lo = x < y ? x : y, hi = x < y ? y : x;
            const bool up = ((8 * l + e) & k) == 0;
            a[e] = up ? lo : hi;
            a[f] = up ? hi : lo;
          }
        }
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e)
    if (8 * l + e < K) row[8 * l + e] = a[e];
}

// Copies each workgroup's staged rows into its contiguous CSR segment with
// unit-stride stores; rows longer than kRowCap are found again and sorted
// in place by their own lane.
__global__ __launch_bounds__(256) void k_nbr_compact(
    const double* __restrict__ xp, int64_t n_mp, double r2, const Grid* __restrict__ gp,
    const int32_t* __restrict__ cell_start, const double4* __restrict__ sorted,
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ stage, int64_t capacity,
    int32_t* __restrict__ idx, int32_t* __restrict__ block_max) {
  __shared__ __align__(16) int32_t rows[kScanMPs * kRowCap];
  __shared__ uint8_t owner[kScanMPs * kRowCap];  // MP of each output element
  __shared__ int64_t off[kScanMPs + 1];
  __shared__ int32_t blk_max;
  const int tid = threadIdx.x;
  const int64_t blk = xcd_block();
  const int64_t p0 = blk * kScanMPs;
  if (p0 >= n_mp) return;
  const int nloc = (int)(n_mp - p0 < kScanMPs ? n_mp - p0 : kScanMPs);
  // every global input is requested before any is used (one memory latency
  // instead of three in a row): the row starts, the total and the staged rows,
  // these in 16-byte pieces (a workgroup's rows start at a multiple of
  // kScanMPs * kRowCap * 4 bytes, and a row's kRowCap ids fill whole pieces)
  static_assert(kScanMPs < 256, "one row start per thread");
  static_assert(kRowCap % 4 == 0, "rows of whole 16-byte pieces");
  constexpr int kPieces = kScanMPs * kRowCap / 4;
  constexpr int kPer = (kPieces + 255) / 256;
  const int64_t my_off = tid <= nloc ? offsets[p0 + tid] : 0;
  const int64_t total_pairs = offsets[n_mp];
  const int4* __restrict__ st4 = reinterpret_cast<const int4*>(stage + p0 * kRowCap);
  int4* rows4 = reinterpret_cast<int4*>(rows);
  const int npc = nloc * (kRowCap / 4);
  int4 st[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = k * 256 + tid;
    st[k] = i < npc ? st4[i] : make_int4(0, 0, 0, 0);
  }
  if (tid <= nloc) off[tid] = my_off;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = k * 256 + tid;
    if (i < npc) rows4[i] = st[k];
  }
  __syncthreads();
  // largest support of the workgroup (reduced once more by k_search_done;
  // one atomic per MP on a single counter would serialise the pass)
  if (tid < kWave) {
    int32_t m = 0;
    for (int i = tid; i < nloc; i += kWave) {
      const int32_t K = (int32_t)(off[i + 1] - off[i]);
      m = K > m ? K : m;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
      const int32_t u = __shfl_xor(m, o);
      m = u > m ? u : m;
    }
    if (tid == 0) {
      block_max[blk] = m;
      blk_max = m;
    }
  }
  if (total_pairs > capacity) return;  // lists do not fit: counts only
  // the staged rows come in stencil order: the four lanes of quad i sort row
  // i (rows past 32 ids, rare, by insertion in LDS in the quad's first lane;
  // rows past kRowCap are re-found below)
  static_assert(4 * kScanMPs == 256, "one quad per staged row");
  if (tid / 4 < nloc) {
    const int i = tid / 4, l = tid % 4;
    const int K = (int)(off[i + 1] - off[i]);
    int32_t* row = rows + i * kRowCap;
    if (K <= 32) {
      sort_row32_quad(row, K, l);
    } else if (K <= kRowCap && l == 0) {
      for (int j = 1; j < K; ++j) {
        const int32_t id = row[j];
        int t = j;
        for (; t > 0 && row[t - 1] > id; --t) row[t] = row[t - 1];
        row[t] = id;
      }
    }
  }
  __syncthreads();
  const int64_t base = off[0];
  const int total = (int)(off[nloc] - base);
  if (blk_max <= kRowCap) {
    // every row is staged: mark the MP of each output element, then copy
    // with unit-stride stores
    for (int t = tid; t < nloc * kRowCap; t += 256) {
      const int i = t / kRowCap, j = t - i * kRowCap;
      if (j < (int)(off[i + 1] - off[i])) owner[(int)(off[i] - base) + j] = (uint8_t)i;
    }
    __syncthreads();
    for (int e = tid; e < total; e += 256) {
      const int i = owner[e];
      idx[base + e] = rows[i * kRowCap + (e - (int)(off[i] - base))];
    }
    return;
  }
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

__global__ __launch_bounds__(1024) void k_search_done(const int64_t* offsets, int64_t n_mp,
                                                      const int32_t* block_max, int64_t nblocks,
                                                      int64_t capacity, otm_diag* diag) {
  __shared__ int32_t red[1024 / kWave];
  // the total is requested first, and the maxima eight at a time, so the
  // loads overlap instead of following one another
  const int64_t P = threadIdx.x == 0 ? offsets[n_mp] : 0;
  int32_t m = 0;
  int64_t b = threadIdx.x;
  for (; b + 7 * 1024 < nblocks; b += 8 * 1024) {
    int32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = block_max[b + k * 1024];
#pragma unroll
    for (int k = 0; k < 8; ++k) m = v[k] > m ? v[k] : m;
  }
  for (; b < nblocks; b += 1024) m = block_max[b] > m ? block_max[b] : m;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int32_t u = __shfl_xor(m, o);
    m = u > m ? u : m;
  }
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x != 0 || diag == nullptr) return;
  for (int w = 1; w < 1024 / kWave; ++w) m = red[w] > m ? red[w] : m;
  diag->pairs_needed = P;
  diag->max_support = m;
  if (P > capacity) atomicOr(&diag->flags, 1u << (-OTM_ERR_CAPACITY - 1));
}

void launch_search(int64_t n_nodes, const double* x_nodes, int64_t n_mp, const double* x_mp,
                   double r_list, double cell_size, int64_t pair_capacity, int64_t* nbr_offsets,
                   int32_t* nbr_idx, const Workspace& w, otm_diag* diag, hipStream_t s) {
  const BinCounters z{w.cell_start, w.cell_cursor, w.mp_cell_start, w.mp_cell_cursor,
                      w.cap_cells};
  k_bbox_partial<<<kBBoxBlocks, 256, 0, s>>>(x_nodes, n_nodes, w.bbox_part, z);
  k_grid_finalize<<<1, 256, 0, s>>>(w.bbox_part, kBBoxBlocks, cell_size, w.cap_cells, w.grid);
  // nodes and MPs binned on the grid together: one count, one two-array scan,
  // one fill
  const BinSet nodes{x_nodes, n_nodes, w.node_cell, w.cell_start, w.cell_cursor, w.sorted};
  const BinSet mps{x_mp, n_mp, w.mp_cell, w.mp_cell_start, w.mp_cell_cursor, w.mp_sorted};
  const int64_t b0 = (n_nodes + kWave - 1) / kWave * kWave;
  const int64_t nt = b0 + n_mp;
  const unsigned nbt = (unsigned)((nt + 255) / 256);
  if (nbt > 0) k_bin_count<<<nbt, 256, 0, s>>>(nodes, mps, b0, w.grid);
  scan_impl<int32_t>(w.cell_start + 1, w.mp_cell_start + 1, w.cap_cells, w.scan_aux, s);
  if (nbt > 0) k_bin_fill<<<nbt, 256, 0, s>>>(nodes, mps, b0);
  const double r2 = r_list * r_list;
  if (n_mp > 0) {
    // a fixed grid (a multiple of the 8 XCDs) strides over the cells
    k_cell_scan<<<kCellBlocks, kCellWaves * kWave, 0, s>>>(r2, w.grid, w.cap_cells, w.cell_start,
                                                   w.sorted, w.mp_cell_start, w.mp_sorted,
                                                   nbr_offsets, w.stage);
    scan_inclusive(nbr_offsets + 1, n_mp, w.scan_aux, s);
    const unsigned nbs = (unsigned)((n_mp + kScanMPs - 1) / kScanMPs);
    k_nbr_compact<<<nbs, 256, 0, s>>>(x_mp, n_mp, r2, w.grid, w.cell_start, w.sorted,
                                      nbr_offsets, w.stage, pair_capacity, nbr_idx,
                                      w.block_max);
  } else {
    k_set_first_offset<<<1, 1, 0, s>>>(nbr_offsets);
  }
  const int64_t nbs_all = (n_mp + kScanMPs - 1) / kScanMPs;
  k_search_done<<<1, 1024, 0, s>>>(nbr_offsets, n_mp, w.block_max, nbs_all, pair_capacity,
                                   diag);
}

}  // namespace otm
