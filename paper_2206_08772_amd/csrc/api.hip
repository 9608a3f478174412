// C ABI of libotm: argument checks, workspace layout and the launch sequence
// of each entry point on the caller's stream.
#include <math.h>
#include <string.h>

#include <mutex>

#include "erode.h"
#include "launch.h"
#include "otm_common.h"

namespace otm {

static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

size_t carve_workspace(void* base, size_t bytes, int64_t n_nodes, int64_t n_mp,
                       int64_t pair_capacity, Workspace* w) {
  const int64_t cap_cells = (n_nodes > 0 ? n_nodes : 0) + 1024;
  // block totals of the largest scan: the MP offsets, the node influence
  // offsets, or the node and MP cell counts scanned together (two arrays)
  auto blocks = [](int64_t n) { return (n + kScanBlock - 1) / kScanBlock; };
  int64_t scan_blocks = blocks(n_mp + 1);
  if (2 * blocks(cap_cells + 1) > scan_blocks) scan_blocks = 2 * blocks(cap_cells + 1);
  if (blocks(n_nodes + 1) > scan_blocks) scan_blocks = blocks(n_nodes + 1);
  scan_blocks += 1;
  const size_t sizes[] = {
      align256(sizeof(Grid)),
      align256(sizeof(double) * 6 * kBBoxBlocks),
      align256(sizeof(int32_t) * (cap_cells + 1)),
      align256(sizeof(int32_t) * cap_cells),
      align256(sizeof(int32_t) * (size_t)n_nodes),
      align256(sizeof(double4) * (size_t)n_nodes),
      align256(sizeof(int64_t) * (size_t)scan_blocks),
      align256(sizeof(int32_t) * (size_t)(n_mp / 64 + 2)),
      align256(sizeof(int64_t) * (size_t)(n_nodes + 1)),
      align256(sizeof(int32_t) * (size_t)n_nodes),
      align256(sizeof(int32_t) * (size_t)pair_capacity),
      align256(sizeof(int32_t) * (size_t)pair_capacity),
      align256(sizeof(int32_t) * (size_t)kRowCapacity * (size_t)n_mp),
      align256(sizeof(double4) * 2 * (size_t)n_nodes),
      align256(sizeof(int32_t) * (cap_cells + 1)),
      align256(sizeof(int32_t) * (size_t)n_mp),
      align256(sizeof(double4) * (size_t)n_mp),
      align256(sizeof(double4) * (size_t)pair_capacity),
      align256(sizeof(int32_t) * cap_cells),
  };
  size_t total = 0;
  for (size_t s : sizes) total += s;
  if (base == nullptr || bytes < total || w == nullptr) return total;
  char* c = (char*)base;
  size_t o = 0;
  auto take = [&](int k) { void* r = c + o; o += sizes[k]; return r; };
  w->grid = (Grid*)take(0);
  w->bbox_part = (double*)take(1);
  w->cap_cells = cap_cells;
  w->cell_start = (int32_t*)take(2);
  w->cell_cursor = (int32_t*)take(3);
  w->node_cell = (int32_t*)take(4);
  w->sorted = (double4*)take(5);
  w->scan_aux = (int64_t*)take(6);
  w->block_max = (int32_t*)take(7);
  w->tr_start = (int64_t*)take(8);
  w->tr_cursor = (int32_t*)take(9);
  w->tr_pairs = (int32_t*)take(10);
  w->tr_pos = (int32_t*)take(11);
  w->stage = (int32_t*)take(12);
  w->nodes = (double4*)take(13);
  w->mp_cell_start = (int32_t*)take(14);
  w->mp_cell = (int32_t*)take(15);
  w->mp_sorted = (double4*)take(16);
  w->contrib = (double4*)take(17);
  w->mp_cell_cursor = (int32_t*)take(18);
  return total;
}

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }
static bool dev_ok(const void* p, size_t a) { return p != nullptr && aligned(p, a); }

static otm_status hip_status() {
  return hipGetLastError() == hipSuccess ? OTM_OK : OTM_ERR_HIP;
}

static otm_status check_workspace(void* ws, size_t ws_bytes, int64_t n_nodes, int64_t n_mp,
                                  int64_t cap, Workspace* w) {
  if (ws == nullptr || !aligned(ws, 256)) return OTM_ERR_ARG;
  const size_t need = carve_workspace(nullptr, 0, n_nodes, n_mp, cap, nullptr);
  if (ws_bytes < need) return OTM_ERR_ARG;
  carve_workspace(ws, ws_bytes, n_nodes, n_mp, cap, w);
  return OTM_OK;
}

static otm_status check_params(const otm_params* p) {
  if (p == nullptr) return OTM_ERR_ARG;
  if (p->model < OTM_NEOHOOKE || p->model > OTM_J2_LINEAR) return OTM_ERR_ARG;
  if (!(p->r_list > 0) || !(p->cell_size >= p->r_list) || !(p->beta > 0)) return OTM_ERR_ARG;
  if (!(p->lme_tol > 0) || p->lme_max_iter < 1 || p->rm_max_iter < 1) return OTM_ERR_ARG;
  if (!(p->E > 0) || !(p->nu > -1.0 && p->nu < 0.5) || !(p->rho0 > 0)) return OTM_ERR_ARG;
  if (!(p->eps_stab >= 0.0) || !isfinite(p->eps_stab)) return OTM_ERR_ARG;
  if (p->body_force[0] != 0.0 || p->body_force[1] != 0.0 || p->body_force[2] != 0.0)
    return OTM_ERR_ARG;
  if (p->model == OTM_J2_JC && !(p->T_m > p->T_r && p->Cp > 0 && p->eps_dot0 > 0))
    return OTM_ERR_ARG;
  if (p->wall_enabled) {
    const double nn = p->wall_n[0] * p->wall_n[0] + p->wall_n[1] * p->wall_n[1] +
                      p->wall_n[2] * p->wall_n[2];
    if (!(fabs(nn - 1.0) < 1e-12)) return OTM_ERR_ARG;
  }
  if (p->fracture != 0 && p->fracture != 1) return OTM_ERR_ARG;
  if (p->fracture) {
    if (p->model != OTM_J2_JC) return OTM_ERR_ARG;
    for (int k = 0; k < 5; ++k)
      if (!isfinite(p->jc_d[k])) return OTM_ERR_ARG;
  }
  if (!(p->kappa >= 0.0) || !isfinite(p->kappa)) return OTM_ERR_ARG;
  if (!(p->insert_dist >= 0.0) || !isfinite(p->insert_dist)) return OTM_ERR_ARG;
  if (p->delete_orphans != 0 && p->delete_orphans != 1) return OTM_ERR_ARG;
  if (p->kappa > 0.0 && (p->model != OTM_J2_JC || p->eps_stab > 0.0)) return OTM_ERR_ARG;
  if (p->tool_enabled != 0 && p->tool_enabled != 1) return OTM_ERR_ARG;
  if (p->tool_enabled) {
    for (int k = 0; k < 3; ++k)
      if (!isfinite(p->tool_c[k]) || !isfinite(p->tool_v[k])) return OTM_ERR_ARG;
    if (!(p->tool_r > 0) || !isfinite(p->tool_r)) return OTM_ERR_ARG;
    if (!(p->tool_clearance >= 0.0 && p->tool_clearance < 1.5707963267948966))
      return OTM_ERR_ARG;
    if (!(p->tool_cN > 0) || !(p->tool_cT > 0) || !isfinite(p->tool_cN) ||
        !isfinite(p->tool_cT) || !(p->tool_mu >= 0) || !isfinite(p->tool_mu))
      return OTM_ERR_ARG;
  }
  return OTM_OK;
}

// The chip-formation and conduction arrays a state needs for these
// parameters (conduction also needs the atomic assembly).
static otm_status check_cut_state(const otm_state* st, const otm_params* p,
                                  int32_t scatter_mode) {
  if (p->fracture && st->n_mp > 0 && !dev_ok(st->failed, 4)) return OTM_ERR_ARG;
  if (p->tool_enabled && (!dev_ok(st->clock, 8) || (st->n_nodes > 0 && !dev_ok(st->tool_gt, 8))))
    return OTM_ERR_ARG;
  if (p->kappa > 0.0) {
    if (scatter_mode != OTM_SCATTER_ATOMIC) return OTM_ERR_ARG;
    if (st->n_nodes > 0 && !dev_ok(st->heat, 8)) return OTM_ERR_ARG;
    if (st->n_mp > 0 && !dev_ok(st->qflux, 8)) return OTM_ERR_ARG;
  }
  return OTM_OK;
}

static otm_status check_state(const otm_state* st) {
  if (st == nullptr) return OTM_ERR_ARG;
  if (st->n_nodes < 0 || st->n_mp < 0 || st->pair_capacity < 0) return OTM_ERR_ARG;
  if (st->pair_capacity >= (int64_t(1) << 31)) return OTM_ERR_ARG;  // int32 pair ids
  if (st->n_nodes >= (int64_t(1) << 31) || st->n_mp >= (int64_t(1) << 31)) return OTM_ERR_ARG;
  if (st->precision != OTM_FP64 && st->precision != OTM_MIXED &&
      st->precision != OTM_MIXED_STORAGE)
    return OTM_ERR_ARG;
  const size_t rs = st->precision == OTM_FP64 ? 8 : 4;
  if (!dev_ok(st->x, 8) || !dev_ok(st->du, 8) || !dev_ok(st->m, 8) || !dev_ok(st->f, 8))
    return OTM_ERR_ARG;
  if (!dev_ok(st->xp, 8) || !dev_ok(st->vol, 8) || !dev_ok(st->mass, 8) ||
      !dev_ok(st->lam, 8) || !dev_ok(st->epsbar, 8) || !dev_ok(st->T, 8))
    return OTM_ERR_ARG;
  if (!dev_ok(st->Fd, rs) || !dev_ok(st->bed, rs) || !dev_ok(st->sigma, rs) ||
      !dev_ok(st->dN, rs))
    return OTM_ERR_ARG;
  if (!dev_ok(st->nbr_offsets, 8) || !dev_ok(st->nbr_idx, 4) || !dev_ok(st->N, 8))
    return OTM_ERR_ARG;
  return OTM_OK;
}

static void mark(hipEvent_t* ev, int k, hipStream_t s) {
  if (ev != nullptr && ev[k] != nullptr) (void)hipEventRecord(ev[k], s);
}

// search (optional) + shape functions + mass/force assembly
// (packed: the node records in the workspace are current; stab: add the
// stabilisation term, which needs the history the MP update just wrote;
// tr: build the segmented mode's influence lists from the current support
// lists even without a search, when the workspace does not hold them)
static void refresh_impl(otm_state& st, const otm_params& p, bool rebuild, int32_t mode,
                         const Workspace& w, otm_diag* diag, hipStream_t s,
                         hipEvent_t* ev = nullptr, bool packed = false, bool stab = false,
                         bool tr = false) {
  const Stab sb = stab ? Stab{p.eps_stab, w.nodes, st.xp, st.xp_prev, st.dFm1}
                       : Stab{0.0, nullptr, nullptr, nullptr, nullptr};
  if (!packed) launch_pack_nodes(st, w.nodes, s);
  if (rebuild)
    launch_search(st.n_nodes, st.x, st.n_mp, st.xp, p.r_list, p.cell_size, st.pair_capacity,
                  st.nbr_offsets, st.nbr_idx, w, diag, s);
  mark(ev, 3, s);
  // Without the stabilisation term the assembly's per-pair work runs inside
  // the shape-function kernel, on N and grad N while they are in registers:
  // the atomic mode sums into LDS node tables there; the segmented mode
  // stores each pair's contributions in node order there (its influence
  // lists, which depend only on the support lists, are built first) and a
  // last kernel sums each node's run.  Events (profiled step): atomic
  // 3 | LME + assembly | 4 | 6; segmented 3 | influence lists | 4 | LME +
  // contributions | 5 | node sums | 6; with the stabilisation term 3 | LME |
  // 4 | assembly (atomic), or 4 | lists | 5 | contributions + sums (segmented) | 6.
  const bool fuse_atomic = mode == OTM_SCATTER_ATOMIC && !stab;
  const bool fuse_seg = mode == OTM_SCATTER_SEGMENTED && !stab;
  // with conduction (atomic mode only) the fused assembly also sums h_I, Q_I
  const bool heat = p.kappa > 0.0;
  if (fuse_seg) {
    if (rebuild || tr) launch_influence_lists(st, w, s);
    mark(ev, 4, s);
  }
  const AsmIn fused{st.vol, st.mass, st.sigma, st.m, st.f, st.n_nodes,
                    heat ? st.T : nullptr, heat ? st.qflux : nullptr, heat ? st.heat : nullptr};
  const SegIn seg{st.vol, st.mass, st.sigma, w.tr_pos, w.contrib};
  launch_lme(st.n_nodes, st.x, st.n_mp, st.xp, st.nbr_offsets, st.nbr_idx, st.pair_capacity,
             p.beta, p.lme_tol, p.lme_max_iter, st.lam, st.N, st.dN, st.precision, w.nodes, diag,
             s, fuse_atomic ? &fused : nullptr, fuse_seg ? &seg : nullptr);
  if (fuse_seg) {
    mark(ev, 5, s);
    launch_seg_gather(st, w, s);
  } else {
    mark(ev, 4, s);
    if (mode == OTM_SCATTER_ATOMIC) {
      if (!fuse_atomic) launch_assemble_atomic(st, sb, s);
    } else {
      if (rebuild || tr) launch_influence_lists(st, w, s);
      mark(ev, 5, s);
      launch_scatter_segmented(st, w, sb, s);
    }
  }
  mark(ev, 6, s);
}

}  // namespace otm

using namespace otm;

extern "C" {

const char* otm_status_string(otm_status s) {
  switch (s) {
    case OTM_OK: return "OTM_OK";
    case OTM_ERR_ARG: return "OTM_ERR_ARG: invalid argument";
    case OTM_ERR_CAPACITY: return "OTM_ERR_CAPACITY: more support pairs than pair_capacity";
    case OTM_ERR_LME_NOCONV: return "OTM_ERR_LME_NOCONV: LME Newton did not converge";
    case OTM_ERR_RM_NOCONV: return "OTM_ERR_RM_NOCONV: return map did not converge";
    case OTM_ERR_INVERTED: return "OTM_ERR_INVERTED: det(dF) <= 0 at a material point";
    case OTM_ERR_NONFINITE: return "OTM_ERR_NONFINITE: non-finite stress or position";
    case OTM_ERR_HIP: return "OTM_ERR_HIP: HIP runtime error";
    case OTM_ERR_SUPPORT: return "OTM_ERR_SUPPORT: support longer than the adjoint handles";
    case OTM_ERR_SCRATCH:
      return "OTM_ERR_SCRATCH: the state needs more scratch than otm_step_noalloc has";
    default: return "unknown otm_status";
  }
}

size_t otm_workspace_bytes(int64_t n_nodes, int64_t n_mp, int64_t pair_capacity) {
  if (n_nodes < 0 || n_mp < 0 || pair_capacity < 0) return 0;
  return carve_workspace(nullptr, 0, n_nodes, n_mp, pair_capacity, nullptr);
}

otm_status otm_diag_reset(otm_diag* diag, hipStream_t s) {
  if (!dev_ok(diag, 8)) return OTM_ERR_ARG;
  launch_diag_reset(diag, s);
  return hip_status();
}

otm_status otm_diag_read(const otm_diag* diag, otm_diag* host_out, hipStream_t s) {
  if (!dev_ok(diag, 8) || host_out == nullptr) return OTM_ERR_ARG;
  if (hipMemcpyAsync(host_out, diag, sizeof(otm_diag), hipMemcpyDeviceToHost, s) != hipSuccess)
    return OTM_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return OTM_ERR_HIP;
  for (int k = 0; k < 8; ++k)
    if (host_out->flags & (1u << k)) return (otm_status)(-(k + 1));
  return OTM_OK;
}

otm_status otm_build_neighbors(int64_t n_nodes, const double* x_nodes, int64_t n_mp,
                               const double* x_mp, double r_list, double cell_size,
                               int64_t pair_capacity, int64_t* nbr_offsets, int32_t* nbr_idx,
                               int64_t* n_pairs_out, void* ws, size_t ws_bytes, hipStream_t s) {
  if (n_nodes < 0 || n_mp < 0 || pair_capacity < 0 || n_pairs_out == nullptr) return OTM_ERR_ARG;
  if (pair_capacity >= (int64_t(1) << 31) || n_nodes >= (int64_t(1) << 31)) return OTM_ERR_ARG;
  if (!(r_list > 0) || !(cell_size >= r_list)) return OTM_ERR_ARG;
  if ((n_nodes > 0 && !dev_ok(x_nodes, 8)) || (n_mp > 0 && !dev_ok(x_mp, 8)) ||
      !dev_ok(nbr_offsets, 8) || (pair_capacity > 0 && !dev_ok(nbr_idx, 4)))
    return OTM_ERR_ARG;
  Workspace w;
  if (check_workspace(ws, ws_bytes, n_nodes, n_mp, pair_capacity, &w) != OTM_OK) return OTM_ERR_ARG;
  if (n_nodes == 0) {
    // no nodes: every support is empty
    launch_fill_i64(nbr_offsets, n_mp + 1, 0, s);
    *n_pairs_out = 0;
    return hipStreamSynchronize(s) == hipSuccess ? hip_status() : OTM_ERR_HIP;
  }
  launch_search(n_nodes, x_nodes, n_mp, x_mp, r_list, cell_size, pair_capacity, nbr_offsets,
                nbr_idx, w, nullptr, s);
  if (hip_status() != OTM_OK) return OTM_ERR_HIP;
  int64_t P = 0;
  if (hipMemcpyAsync(&P, nbr_offsets + n_mp, sizeof(int64_t), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return OTM_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return OTM_ERR_HIP;
  *n_pairs_out = P;
  return P > pair_capacity ? OTM_ERR_CAPACITY : OTM_OK;
}

otm_status otm_lme_shape(int64_t n_nodes, const double* x_nodes, int64_t n_mp,
                         const double* x_mp, const int64_t* nbr_offsets, const int32_t* nbr_idx,
                         int64_t pair_capacity, double beta, double tol, int32_t max_iter,
                         double* lam, double* N, void* dN, int32_t precision, otm_diag* diag,
                         hipStream_t s) {
  if (n_nodes < 0 || n_mp < 0 || pair_capacity < 0) return OTM_ERR_ARG;
  if (!(beta > 0) || !(tol > 0) || max_iter < 1) return OTM_ERR_ARG;
  if (precision != OTM_FP64 && precision != OTM_MIXED && precision != OTM_MIXED_STORAGE)
    return OTM_ERR_ARG;
  const size_t rs = precision == OTM_FP64 ? 8 : 4;
  if (n_mp == 0) return OTM_OK;
  if (!dev_ok(x_nodes, 8) || !dev_ok(x_mp, 8) || !dev_ok(nbr_offsets, 8) || !dev_ok(lam, 8))
    return OTM_ERR_ARG;
  if (pair_capacity > 0 && (!dev_ok(nbr_idx, 4) || !dev_ok(N, 8) || !dev_ok(dN, rs)))
    return OTM_ERR_ARG;
  if (diag != nullptr && !aligned(diag, 8)) return OTM_ERR_ARG;
  launch_lme(n_nodes, x_nodes, n_mp, x_mp, nbr_offsets, nbr_idx, pair_capacity, beta, tol,
             max_iter, lam, N, dN, precision, nullptr, diag, s);
  return hip_status();
}

otm_status otm_refresh(otm_state* st, const otm_params* p, int32_t rebuild, int32_t scatter_mode,
                       void* ws, size_t ws_bytes, otm_diag* diag, hipStream_t s) {
  otm_status e;
  if ((e = check_state(st)) != OTM_OK || (e = check_params(p)) != OTM_OK) return e;
  if (scatter_mode != OTM_SCATTER_ATOMIC && scatter_mode != OTM_SCATTER_SEGMENTED)
    return OTM_ERR_ARG;
  if (!dev_ok(diag, 8)) return OTM_ERR_ARG;
  Workspace w;
  if (check_workspace(ws, ws_bytes, st->n_nodes, st->n_mp, st->pair_capacity, &w) != OTM_OK)
    return OTM_ERR_ARG;
  if ((e = check_cut_state(st, p, scatter_mode)) != OTM_OK) return e;
  if (scatter_mode == OTM_SCATTER_ATOMIC) {
    launch_zero(st->m, st->n_nodes, s);
    launch_zero(st->f, 3 * st->n_nodes, s);
    if (p->kappa > 0.0) launch_zero(st->heat, 2 * st->n_nodes, s);
  }
  // the influence lists are rebuilt from the lists as they are: a caller
  // may have replaced them (a resumed run) since the workspace last saw them
  refresh_impl(*st, *p, rebuild != 0, scatter_mode, w, diag, s, nullptr, false, false, true);
  return hip_status();
}

otm_status otm_init(otm_state* st, const otm_params* p, double dt, const double* v0,
                    int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                    hipStream_t s) {
  otm_status e;
  if ((e = check_state(st)) != OTM_OK || (e = check_params(p)) != OTM_OK) return e;
  if (!(dt > 0) || (st->n_nodes > 0 && !dev_ok(v0, 8))) return OTM_ERR_ARG;
  if ((e = check_cut_state(st, p, scatter_mode)) != OTM_OK) return e;
  launch_init_fields(*st, *p, dt, v0, s);
  return otm_refresh(st, p, 1, scatter_mode, ws, ws_bytes, diag, s);
}

static otm_status step_impl(otm_state* st, const otm_params* p, double dt, int32_t rebuild,
                            int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                            hipEvent_t* ev, hipStream_t s, const otm_lists* next = nullptr,
                            bool tr = false) {
  otm_status e;
  if ((e = check_state(st)) != OTM_OK || (e = check_params(p)) != OTM_OK) return e;
  if (next != nullptr) {
    const size_t rs = st->precision == OTM_FP64 ? 8 : 4;
    if (!dev_ok(next->nbr_offsets, 8) || !dev_ok(next->nbr_idx, 4) || !dev_ok(next->N, 8) ||
        !dev_ok(next->dN, rs))
      return OTM_ERR_ARG;
    if (next->nbr_offsets == st->nbr_offsets || next->nbr_idx == st->nbr_idx ||
        next->N == st->N || next->dN == st->dN)
      return OTM_ERR_ARG;
  }
  if (!(dt > 0)) return OTM_ERR_ARG;
  if (scatter_mode != OTM_SCATTER_ATOMIC && scatter_mode != OTM_SCATTER_SEGMENTED)
    return OTM_ERR_ARG;
  if (!dev_ok(diag, 8)) return OTM_ERR_ARG;
  const bool stab = p->eps_stab > 0.0;
  if (stab && (!dev_ok(st->xp_prev, 8) || !dev_ok(st->dFm1, 8))) return OTM_ERR_ARG;
  if ((e = check_cut_state(st, p, scatter_mode)) != OTM_OK) return e;
  Workspace w;
  if (check_workspace(ws, ws_bytes, st->n_nodes, st->n_mp, st->pair_capacity, &w) != OTM_OK)
    return OTM_ERR_ARG;
  mark(ev, 0, s);
  launch_node_update(*st, *p, dt, scatter_mode == OTM_SCATTER_ATOMIC, w.nodes, diag, s);
  mark(ev, 1, s);
  launch_mp_update(*st, *p, dt, w.nodes, diag, s);
  mark(ev, 2, s);
  if (next == nullptr) {
    refresh_impl(*st, *p, rebuild != 0, scatter_mode, w, diag, s, ev, true, stab, tr);
    return hip_status();
  }
  otm_state to = *st;
  to.nbr_offsets = next->nbr_offsets;
  to.nbr_idx = next->nbr_idx;
  to.N = next->N;
  to.dN = next->dN;
  if (rebuild == 0) {  // the lists of step n carry over
    if (hipMemcpyAsync(to.nbr_offsets, st->nbr_offsets, sizeof(int64_t) * (size_t)(st->n_mp + 1),
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return OTM_ERR_HIP;
    if (st->pair_capacity > 0 &&
        hipMemcpyAsync(to.nbr_idx, st->nbr_idx, sizeof(int32_t) * (size_t)st->pair_capacity,
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
      return OTM_ERR_HIP;
  }
  refresh_impl(to, *p, rebuild != 0, scatter_mode, w, diag, s, ev, true, stab, tr);
  if ((e = hip_status()) != OTM_OK) return e;
  *st = to;
  return OTM_OK;
}

otm_status otm_step(otm_state* st, const otm_params* p, double dt, int32_t rebuild,
                    int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                    hipStream_t s) {
  return step_impl(st, p, dt, rebuild, scatter_mode, ws, ws_bytes, diag, nullptr, s);
}

otm_status otm_step_into(otm_state* st, const otm_lists* next, const otm_params* p, double dt,
                         int32_t rebuild, int32_t scatter_mode, void* ws, size_t ws_bytes,
                         otm_diag* diag, hipStream_t s) {
  if (next == nullptr) return OTM_ERR_ARG;
  return step_impl(st, p, dt, rebuild, scatter_mode, ws, ws_bytes, diag, nullptr, s, next);
}

otm_status otm_step_profiled(otm_state* st, const otm_params* p, double dt, int32_t rebuild,
                             int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                             hipEvent_t* events, hipStream_t s) {
  if (events == nullptr) return OTM_ERR_ARG;
  return step_impl(st, p, dt, rebuild, scatter_mode, ws, ws_bytes, diag, events, s);
}

}  // extern "C"

// Allocation-free step: the workspace is this file-scope device array.  Each
// device holds its own copy at its own address, found once per device with
// hipGetSymbolAddress; host code only ever passes that address on (the
// array's name in host code is a stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[OTM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kMaxDevices] = {};

static otm_status static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return OTM_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
      return OTM_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return OTM_OK;
}

extern "C" {

otm_status otm_step_noalloc(otm_state* st, const otm_params* p, double dt, int32_t rebuild,
                            int32_t scatter_mode, otm_diag* diag, hipStream_t s) {
  otm_status e;
  if ((e = check_state(st)) != OTM_OK || (e = check_params(p)) != OTM_OK) return e;
  if (carve_workspace(nullptr, 0, st->n_nodes, st->n_mp, st->pair_capacity, nullptr) >
      (size_t)OTM_STATIC_SCRATCH_BYTES)
    return OTM_ERR_SCRATCH;
  void* ws = nullptr;
  if ((e = static_scratch(&ws)) != OTM_OK) return e;
  // the scratch holds whatever the last call on this device left: the
  // segmented mode's influence lists are built anew from the state's lists
  return step_impl(st, p, dt, rebuild, scatter_mode, ws, (size_t)OTM_STATIC_SCRATCH_BYTES,
                   diag, nullptr, s, nullptr, true);
}

otm_status otm_erode(otm_state* st, const otm_params* p, int32_t scatter_mode, void* ws,
                     size_t ws_bytes, otm_diag* diag, int64_t* n_removed, int64_t* node_events,
                     hipStream_t s) {
  otm_status e;
  if ((e = check_state(st)) != OTM_OK || (e = check_params(p)) != OTM_OK) return e;
  if (n_removed == nullptr || !p->fracture || p->eps_stab > 0.0) return OTM_ERR_ARG;
  if (scatter_mode != OTM_SCATTER_ATOMIC && scatter_mode != OTM_SCATTER_SEGMENTED)
    return OTM_ERR_ARG;
  if (!dev_ok(diag, 8)) return OTM_ERR_ARG;
  if ((e = check_cut_state(st, p, scatter_mode)) != OTM_OK) return e;
  if (st->node_capacity < 0 || st->node_capacity >= (int64_t(1) << 31)) return OTM_ERR_ARG;
  // nodes may be added up to the capacity: the workspace is laid out for it
  const int64_t ncap = st->node_capacity > st->n_nodes ? st->node_capacity : st->n_nodes;
  Workspace w;
  if (check_workspace(ws, ws_bytes, ncap, st->n_mp, st->pair_capacity, &w) != OTM_OK)
    return OTM_ERR_ARG;
  const int64_t n0 = st->n_mp;
  int64_t inserted = 0, deleted = 0;
  otm_state to = *st;
  if ((e = launch_erode(to, *p, w, s, &inserted)) != OTM_OK) return e;
  st->n_mp = to.n_mp;
  st->n_nodes = to.n_nodes;
  *n_removed = n0 - to.n_mp;
  // lists, shape functions, mass and force of the remaining body
  if ((e = otm_refresh(st, p, 1, scatter_mode, ws, ws_bytes, diag, s)) != OTM_OK) return e;
  if (p->delete_orphans) {
    if ((e = launch_delete_orphans(*st, *p, w, s, &deleted)) != OTM_OK) return e;
    if (deleted > 0 && scatter_mode == OTM_SCATTER_SEGMENTED) {
      // the next step's influence lists, in the layout of its workspace
      Workspace wn;
      carve_workspace(ws, ws_bytes, st->n_nodes, st->n_mp, st->pair_capacity, &wn);
      launch_influence_lists(*st, wn, s);
    }
  }
  if (node_events != nullptr) {
    node_events[0] = inserted;
    node_events[1] = deleted;
  }
  return hip_status();
}

size_t otm_adjoint_workspace_bytes(int64_t n_nodes, int64_t n_mp) {
  if (n_nodes < 0 || n_mp < 0) return 0;
  return adjoint_workspace_bytes(n_nodes, n_mp);
}

static bool tape_ok(const otm_tape* t) {
  if (t == nullptr || t->n_nodes < 0 || t->n_mp < 0 || t->pair_stride < 0) return false;
  const void* p8[] = {t->x, t->du, t->m, t->f, t->xp, t->vol, t->lam, t->Fd, t->bed,
                      t->epsbar, t->T, t->sigma, t->nbr_offsets, t->N, t->dN};
  for (const void* q : p8)
    if (!dev_ok(q, 8)) return false;
  return dev_ok(t->nbr_idx, 4);
}

static bool bar_ok(const otm_state_bar* b) {
  if (b == nullptr) return false;
  const void* p8[] = {b->x, b->du, b->vol, b->Fd, b->bed, b->epsbar, b->T, b->sigma, b->N, b->dN};
  for (const void* q : p8)
    if (!dev_ok(q, 8)) return false;
  return true;
}

otm_status otm_init_adjoint(int64_t n_nodes, double dt, const double* du_bar, double* v0_bar,
                            const double* dir, double* dir_bar, hipStream_t s) {
  if (n_nodes < 0 || !(dt > 0) || !isfinite(dt)) return OTM_ERR_ARG;
  if (n_nodes > 0 && (!dev_ok(du_bar, 8) || !dev_ok(v0_bar, 8))) return OTM_ERR_ARG;
  if ((dir == nullptr) != (dir_bar == nullptr)) return OTM_ERR_ARG;
  if (dir_bar != nullptr && (!dev_ok(dir_bar, 8) || (n_nodes > 0 && !dev_ok(dir, 8))))
    return OTM_ERR_ARG;
  if (n_nodes > 0 && (du_bar == v0_bar || (dir != nullptr && dir == v0_bar))) return OTM_ERR_ARG;
  launch_init_adjoint(n_nodes, dt, du_bar, v0_bar, dir, dir_bar, s);
  return hip_status();
}

otm_status otm_step_adjoint(const otm_tape* tn, const otm_tape* tn1, const otm_params* p,
                            double dt, const double* mass, otm_state_bar* bar_next,
                            otm_state_bar* bar, double* theta_bar, void* ws, size_t ws_bytes,
                            otm_diag* diag, hipStream_t s) {
  otm_status e;
  if ((e = check_params(p)) != OTM_OK) return e;
  if (p->model == OTM_NEOHOOKE) return OTM_ERR_ARG;  // adjoint covers the J2 models
  if (p->eps_stab != 0.0) return OTM_ERR_ARG;        // no adjoint of the stabilisation
  if (p->fracture || p->tool_enabled) return OTM_ERR_ARG;  // nor of fracture and the tool
  if (p->kappa > 0.0) return OTM_ERR_ARG;                  // nor of heat conduction
  if (!tape_ok(tn) || !tape_ok(tn1) || !bar_ok(bar_next) || !bar_ok(bar)) return OTM_ERR_ARG;
  if (tn->n_nodes != tn1->n_nodes || tn->n_mp != tn1->n_mp) return OTM_ERR_ARG;
  if (!(dt > 0) || !dev_ok(mass, 8) || !dev_ok(theta_bar, 8) || !dev_ok(diag, 8))
    return OTM_ERR_ARG;
  if (ws == nullptr || !aligned(ws, 256) ||
      ws_bytes < adjoint_workspace_bytes(tn->n_nodes, tn->n_mp))
    return OTM_ERR_ARG;
  launch_step_adjoint(*tn, *tn1, *p, dt, mass, *bar_next, *bar, theta_bar, ws, diag, s);
  return hip_status();
}

}  // extern "C"
