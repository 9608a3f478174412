// Internal host-side launchers and workspace layout of libotm (not exported).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "otm.h"

namespace otm {

// Linked-cell grid parameters, computed on the device from the node bounding
// box so that no host round trip is needed.
struct Grid {
  double lo[3];
  double cell;
  int32_t dims[3];
  int32_t pad;
  int64_t n_cells;
};

constexpr int kBBoxBlocks = 256;
constexpr int kScanBlock = 4096;  // elements per scan workgroup (1024 threads x 4)
constexpr int kRowCapacity = 40;  // search rows staged per MP before compaction

struct Workspace {
  Grid* grid;
  double* bbox_part;     // [kBBoxBlocks][6]
  int64_t cap_cells;
  int32_t* cell_start;   // [cap_cells + 1]
  int32_t* cell_cursor;  // [cap_cells]
  int32_t* node_cell;    // [n_nodes]
  double4* sorted;       // [n_nodes]: x, y, z, node id
  int64_t* scan_aux;     // scan partial sums (int64 view)
  int32_t* block_max;    // [n_mp / 64 + 1] largest support per compaction workgroup
  int64_t* tr_start;     // [n_nodes + 1] influence-list offsets
  int32_t* tr_cursor;    // [n_nodes]
  int32_t* tr_pairs;     // [pair_capacity] pair ids bucketed by node (order within a bucket unset)
  int32_t* tr_pos;       // [pair_capacity] place of each pair in the node-sorted order
  int32_t* stage;        // [n_mp][kRowCapacity] sorted rows of the one-pass search
  double4* nodes;        // [2 n_nodes] packed node records (x, y, z, du_x), (du_y, du_z, 0, 0)
  int32_t* mp_cell_start;  // [cap_cells + 1] MPs binned on the search grid
  int32_t* mp_cell_cursor; // [cap_cells]
  int32_t* mp_cell;        // [n_mp]
  double4* mp_sorted;      // [n_mp]: x, y, z, MP id
  double4* contrib;        // [pair_capacity] pair contributions (m, f) in node-sorted order
};

// Lays the workspace out over [base, base + bytes).  Returns the bytes needed
// (the layout is only written when base != nullptr and bytes suffice).
size_t carve_workspace(void* base, size_t bytes, int64_t n_nodes, int64_t n_mp,
                       int64_t pair_capacity, Workspace* w);

// In-place inclusive prefix sums.
void scan_inclusive(int64_t* a, int64_t n, int64_t* aux, hipStream_t s);
void scan_inclusive(int32_t* a, int64_t n, int64_t* aux, hipStream_t s);

// Search: counts into nbr_offsets, scans, and (fill) writes sorted lists if the
// total fits pair_capacity.  Never synchronises.
void launch_search(int64_t n_nodes, const double* x_nodes, int64_t n_mp, const double* x_mp,
                   double r_list, double cell_size, int64_t pair_capacity, int64_t* nbr_offsets,
                   int32_t* nbr_idx, const Workspace& w, otm_diag* diag, hipStream_t s);

// Inputs of the atomic assembly when it is fused into the shape-function
// kernel (m and f must be zero beforehand; sigma is double or float per the
// precision).  With conduction (heat != nullptr, zero beforehand) it also
// sums h_I = sum N m_p T_p and Q_I = sum v_p q_p . grad N into heat [2][n].
struct AsmIn {
  const double* vol;
  const double* mass;
  const void* sigma;
  double* m;
  double* f;
  int64_t n_nodes;
  const double* T = nullptr;
  const double* q = nullptr;
  double* heat = nullptr;
};

// Inputs of the deterministic assembly's contribution store when it is fused
// into the shape-function kernel (the influence lists must be current).
struct SegIn {
  const double* vol;
  const double* mass;
  const void* sigma;
  const int32_t* pos_of;
  double4* contrib;
};

// LME shape functions (float64 Newton; dN stored per precision).
// ``packed`` (nullable): node records (x, y, z, du_x) at even indices.
// ``fused`` (nullable): also assemble m and f from the new N and grad N.
// ``seg`` (nullable): also store every pair's contributions in node order.
void launch_lme(int64_t n_nodes, const double* x_nodes, int64_t n_mp, const double* x_mp,
                const int64_t* nbr_offsets, const int32_t* nbr_idx, int64_t pair_capacity,
                double beta, double tol, int32_t max_iter, double* lam, double* N, void* dN,
                int32_t precision, const double4* packed, otm_diag* diag, hipStream_t s,
                const AsmIn* fused = nullptr, const SegIn* seg = nullptr);

// Nodes and material points.
// Node records: packed[2 I] = (x, y, z, du_x), packed[2 I + 1] = (du_y, du_z,
// T_I, T_I rate) with conduction (the nodal temperature and its rate from
// st.heat), else (du_y, du_z, 0, 0).
// The MP update also writes the stabilisation history (st.xp_prev, st.dFm1)
// when p.eps_stab > 0.
void launch_node_update(const otm_state& st, const otm_params& p, double dt, bool zero_mf,
                        double4* packed, otm_diag* diag, hipStream_t s);
void launch_pack_nodes(const otm_state& st, double4* packed, hipStream_t s);
void launch_mp_update(const otm_state& st, const otm_params& p, double dt,
                      const double4* packed, otm_diag* diag, hipStream_t s);
void launch_init_fields(const otm_state& st, const otm_params& p, double dt, const double* v0,
                        hipStream_t s);
void launch_zero(double* a, int64_t n, hipStream_t s);
void launch_fill_i32(int32_t* a, int64_t n, int32_t v, hipStream_t s);
void launch_fill_i64(int64_t* a, int64_t n, int64_t v, hipStream_t s);

// Inputs of the stabilisation term -eps sum_p N_Ip e_Ip of the nodal force
// (eps == 0: no term): the node records of this step, the MP positions, and
// the MP positions and dF - 1 before / of the MP update of this step.
struct Stab {
  double eps;
  const double4* nodes;
  const double* xp;
  const double* xp_prev;
  const double* dFm1;
};

// Segmented (deterministic) assembly.
void launch_influence_lists(const otm_state& st, const Workspace& w, hipStream_t s);
void launch_scatter_segmented(const otm_state& st, const Workspace& w, const Stab& sb,
                              hipStream_t s);
// Only the per-node ordered sums (contributions already stored).
void launch_seg_gather(const otm_state& st, const Workspace& w, hipStream_t s);
// Atomic assembly (m and f must be zero beforehand).
void launch_assemble_atomic(const otm_state& st, const Stab& sb, hipStream_t s);

void launch_diag_reset(otm_diag* d, hipStream_t s);

// Adjoint of one step.
size_t adjoint_workspace_bytes(int64_t n_nodes, int64_t n_mp);
void launch_step_adjoint(const otm_tape& t0, const otm_tape& t1, const otm_params& p,
                         double dt, const double* mass, otm_state_bar& b1, otm_state_bar& b0,
                         double* theta_bar, void* ws, otm_diag* diag, hipStream_t s);
// Adjoint of du_0 = dt v0 (and its dot product with a direction).
void launch_init_adjoint(int64_t n_nodes, double dt, const double* du_bar, double* v0_bar,
                         const double* dir, double* dir_bar, hipStream_t s);

}  // namespace otm
