/*
 * otm.h -- C ABI of libotm.so, the explicit step of the Optimal Transportation
 * Meshfree (OTM) method on one AMD Instinct MI355X (gfx950).
 *
 * The step follows Alg. 1 of the paper (Kumar, Gosselet, Huang, Weissenfels,
 * Wriggers, "Parallel multiphysics simulation for the stabilized optimal
 * transportation meshfree (OTM) method"): lumped mass and nodal force,
 * central-difference update of the nodes, material-point (MP) positions and
 * deformation gradients, constitutive update, linked-cell search of the
 * support domains (Alg. 3) and local max-ent (LME) shape functions (Sec. 2.3).
 *
 * Conventions shared by every entry point
 *  - All array arguments are DEVICE pointers into caller-owned buffers, unless
 *    marked "host".  The library never allocates device memory: scratch space
 *    comes from a caller-provided workspace of otm_workspace_bytes() bytes,
 *    256-byte aligned (otm_step_noalloc instead uses a fixed device array of
 *    the library).  The caller keeps ownership of everything it passes.
 *  - Vector fields are structure-of-arrays: a "[3][n]" array holds all x
 *    components, then all y, then all z.  Second-order tensors are stored per
 *    component: F as [9][n] row major (F_ij at component 3*i+j), symmetric
 *    tensors as [6][n] in the order xx, yy, zz, xy, yz, xz.
 *  - Support lists are CSR over MPs: nbr_offsets[n_mp+1] (int64, offsets[0]=0)
 *    and nbr_idx[] (int32 node ids, ascending within each MP).  Per-pair
 *    arrays (N, dN) follow the same pair order; dN is [3][pair_capacity].
 *  - Work is enqueued asynchronously on the caller's HIP stream.  Only
 *    otm_build_neighbors and otm_diag_read synchronise that stream.
 *  - Errors the host can see (null or misaligned pointers, negative sizes,
 *    cell edge below the search radius, unknown enums, workspace too small)
 *    are returned at once and nothing is enqueued.  Errors found on the device
 *    (LME or return-map non-convergence, inverted or non-finite material
 *    points, pair capacity exceeded) are recorded in the caller's device
 *    otm_diag record and reported by otm_diag_read.
 *  - No C++ exception crosses this interface.  The library keeps no state
 *    between calls (but for the per-device address of otm_step_noalloc's
 *    scratch); calls on distinct streams with distinct buffers may run
 *    concurrently (otm_step_noalloc calls on one device may not).
 */
#ifndef OTM_H
#define OTM_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t otm_status;
enum {
  OTM_OK = 0,
  OTM_ERR_ARG = -1,          /* invalid argument (host check) */
  OTM_ERR_CAPACITY = -2,     /* more support pairs than pair_capacity */
  OTM_ERR_LME_NOCONV = -3,   /* LME Newton did not converge */
  OTM_ERR_RM_NOCONV = -4,    /* return-map Newton did not converge */
  OTM_ERR_INVERTED = -5,     /* det(dF) <= 0 at a material point */
  OTM_ERR_NONFINITE = -6,    /* non-finite stress or position */
  OTM_ERR_HIP = -7,          /* a HIP runtime call failed */
  OTM_ERR_SUPPORT = -8,      /* a support longer than the adjoint handles (48) */
  OTM_ERR_SCRATCH = -9       /* otm_step_noalloc: the state needs more scratch
                                than OTM_STATIC_SCRATCH_BYTES (host check) */
};

/* arithmetic of the step */
enum { OTM_FP64 = 0,            /* everything in float64 */
       OTM_MIXED = 1,           /* return map, stress, F, b^e, grad N and force
                                   products in float32; LME Newton, N,
                                   positions, volumes, masses and nodal
                                   accumulation in float64 */
       OTM_MIXED_STORAGE = 2 }; /* F, b^e, stress and grad N stored in float32
                                   (as OTM_MIXED), all arithmetic in float64 */
/* nodal force assembly */
enum { OTM_SCATTER_ATOMIC = 0,      /* contributions summed per node in LDS
                                       by each workgroup, then float64 atomic
                                       adds; order varies from run to run */
       OTM_SCATTER_SEGMENTED = 1 }; /* pairs sorted by node (influence lists),
                                       fixed-order gather: bit-reproducible */
/* constitutive model */
enum { OTM_NEOHOOKE = 0,   /* compressible Neo-Hookean */
       OTM_J2_JC = 1,      /* J2, Hencky, Johnson-Cook + adiabatic heating */
       OTM_J2_LINEAR = 2 };/* J2, Hencky, linear isotropic hardening */

/* Material, search, solver and contact parameters (host struct). */
typedef struct otm_params {
  int32_t model;          /* OTM_NEOHOOKE / OTM_J2_JC / OTM_J2_LINEAR */
  int32_t wall_enabled;   /* rigid frictionless plane on/off */
  double E, nu, rho0;     /* Young's modulus, Poisson ratio, reference density */
  double A, B, n, C, m;   /* Johnson-Cook flow stress constants */
  double eps_dot0;        /* JC reference plastic strain rate */
  double T_r, T_m;        /* JC room and melting temperature */
  double Cp, chi;         /* heat capacity, Taylor-Quinney coefficient */
  double Y0, H;           /* linear hardening: initial yield, modulus */
  double beta;            /* LME locality beta = gamma / h^2 */
  double r_list;          /* support (search) radius, r_cut + skin */
  double cell_size;       /* linked-cell edge, >= r_list */
  double lme_tol;         /* LME stop: |sum N_I (x_p - x_I)|_2 <= lme_tol */
  int32_t lme_max_iter;   /* LME Newton iteration cap */
  int32_t rm_max_iter;    /* return-map Newton iteration cap */
  double rm_tol;          /* return-map relative step / bracket tolerance */
  double wall_x[3];       /* a point of the wall plane */
  double wall_n[3];       /* unit normal of the wall, pointing into the body */
  double eps_stab;        /* stabilisation penalty eps >= 0, a force (0: off).
                             With eps > 0, otm_step adds -eps sum_p N_Ip e_Ip
                             to f (Sec. 2.1, stabilised residual) with
                             e_Ip = [(x_I - x_p) - dF_p (x_I,prev - x_p,prev)]
                             / |x_I,prev - x_p,prev|, x_I,prev = x_I - du_I, and
                             needs st->xp_prev and st->dFm1; otm_init and
                             otm_refresh (no previous configuration) add no
                             term; otm_step_adjoint rejects eps > 0 */
  double body_force[3];   /* specific body force: must be 0 */
  /* Chip formation (Sec. 4.2).  Johnson-Cook fracture: after the return map
     an MP whose equivalent plastic strain is positive and at least
     [d1 + d2 exp(d3 eta)] [1 + d4 ln max(rate / eps_dot0, 1)] [1 + d5 T*]
     (eta = mean / von Mises stress, T* the clamped homologous temperature)
     fails: from then on it carries no stress (it keeps its mass, F and
     position; its b^e, epsbar and T stay as they were).  Needs model
     OTM_J2_JC and st->failed. */
  int32_t fracture;       /* fracture criterion on (1) / off (0) */
  int32_t tool_enabled;   /* rigid cutting tool on (1) / off (0) */
  double jc_d[5];         /* fracture constants d1..d5 */
  /* Rigid tool: a wedge rounded by the tip radius and extruded along z.  Its
     tip circle is centred at tool_c + t tool_v at time t; the rake face runs
     from the tip along +y (rake angle 0), the flank face along
     (cos a, sin a, 0), a = tool_clearance.  Each step the nodes inside it
     (normal gap g < 0 at x_n and the tool at t_n) get the penalty force
     tool_cN |g| along the outward normal plus a tangential force: the trial
     -tool_cT g_T (g_T the node's tangential gap, see otm_state::tool_gt)
     while it is at most tool_mu times the normal force (stick), else that
     limit along it (Coulomb slip).  At a node of lumped mass m both penalty
     stiffnesses are limited to m / dt^2 (one step removes the whole
     penetration; a light node would otherwise make the explicit contact
     unstable), and a node without mass feels none.  The force joins the
     internal force in the node update.  Needs st->tool_gt and st->clock. */
  double tool_c[3];       /* centre of the tip circle at t = 0 */
  double tool_v[3];       /* tool velocity */
  double tool_r;          /* tip radius > 0 */
  double tool_clearance;  /* clearance angle in [0, pi/2) */
  double tool_cN, tool_cT;/* normal and tangential penalty stiffness > 0 (N/m) */
  double tool_mu;         /* Coulomb friction coefficient >= 0 */
  /* Heat conduction (the paper's chip-formation model is adiabatic; this
     adds Fourier conduction q = -kappa grad T through the LME gradients).
     With kappa > 0 each MP update also adds
       dT_p = dt sum_I N_Ip Q_I / (Cp m_I),  Q_I = sum_p v_p q_p . grad N_Ip,
     to T_{n+1} with the plastic heating, where q_p = -kappa sum_I T_I grad N_Ip
     is the flux of the previous MP update (st->qflux) and
     T_I = sum_p N_Ip m_p T_p / m_I the mass-weighted nodal temperature; the
     flow stress still softens with T_n, the fracture check sees T_{n+1}, and
     a failed MP takes its conduction increment too.  The sums h_I and Q_I
     are assembled with the mass and force into st->heat.  The surface is
     insulated.  Needs model OTM_J2_JC, the atomic assembly, eps_stab = 0 and
     st->heat, st->qflux; otm_step_adjoint rejects kappa > 0. */
  double kappa;           /* thermal conductivity >= 0 (0: adiabatic) */
  /* Node management at erosion (otm_erode; the data management of Sec. 3.3
     adds and deletes nodes). */
  double insert_dist;     /* > 0: a removed MP whose support has no node
                             within this distance, and which has no removed
                             MP of smaller index within it, leaves a node at
                             its position (0: no insertion) */
  int32_t delete_orphans; /* 1: nodes in no support after the erosion are
                             removed from the node set (0: they stay) */
  int32_t pad1;
} otm_params;

/* Device state of one simulation (host struct of device pointers). */
typedef struct otm_state {
  int64_t n_nodes, n_mp;
  int64_t pair_capacity;  /* length of nbr_idx and N; dN is [3][pair_capacity].
                             Any value works; an even one (with nbr_idx 8-byte,
                             N 16-byte and dN 16-byte (8-byte if float) aligned)
                             lets the MP update load two pairs at once */
  int32_t precision;      /* OTM_FP64, OTM_MIXED or OTM_MIXED_STORAGE: types of
                             the void* fields (float in both mixed modes) */
  int32_t pad0;
  /* nodes */
  double* x;              /* [3][n_nodes] current positions */
  double* du;             /* [3][n_nodes] displacement increment of the last step */
  double* m;              /* [n_nodes] lumped mass */
  double* f;              /* [3][n_nodes] internal force */
  /* material points */
  double* xp;             /* [3][n_mp] positions */
  double* vol;            /* [n_mp] current volume */
  const double* mass;     /* [n_mp] mass (constant; otm_erode compacts it) */
  double* lam;            /* [3][n_mp] LME multiplier (warm start) */
  void* Fd;               /* [9][n_mp] F - 1 (double, or float in the mixed modes) */
  void* bed;              /* [6][n_mp] b^e - 1 (double / float) */
  double* epsbar;         /* [n_mp] equivalent plastic strain */
  double* T;              /* [n_mp] temperature */
  void* sigma;            /* [6][n_mp] Cauchy stress (double / float) */
  /* support lists and shape functions */
  int64_t* nbr_offsets;   /* [n_mp+1] */
  int32_t* nbr_idx;       /* [pair_capacity] */
  double* N;              /* [pair_capacity] */
  void* dN;               /* [3][pair_capacity] (double / float) */
  /* stabilisation history, written by otm_step's MP update when
     params.eps_stab > 0 (may be NULL otherwise) */
  double* xp_prev;        /* [3][n_mp] MP positions before the last MP update */
  double* dFm1;           /* [9][n_mp] dF - 1 of the last MP update (float64 in
                             both precisions), row-major per MP */
  /* chip formation (may be NULL when params.fracture / tool_enabled are 0) */
  int32_t* failed;        /* [n_mp] 1 once the MP met the fracture criterion */
  double* tool_gt;        /* [3][n_nodes] tangential contact gap of each node:
                             each step in contact it becomes the previous gap,
                             projected on the tangent plane, plus the tangential
                             part of du_I - dt tool_v, cut back to the Coulomb
                             limit (g_T = -t_T / tool_cT); 0 out of contact */
  double* clock;          /* [1] time of the state; otm_init sets 0 and each
                             step adds dt (moves the tool) */
  /* heat conduction (may be NULL when params.kappa is 0) */
  double* heat;           /* [2][n_nodes] h_I = sum_p N_Ip m_p T_p and
                             Q_I = sum_p v_p q_p . grad N_Ip of the last
                             assembly */
  double* qflux;          /* [3][n_mp] heat flux q_p of the last MP update
                             (otm_init sets 0; otm_erode compacts it) */
  int64_t node_capacity;  /* entries per component the node arrays (x, du,
                             m, f, tool_gt, heat) have room for, >= n_nodes
                             (0: n_nodes); otm_erode adds nodes up to it */
} otm_state;

/* Device-side failure record (lives in device memory). */
typedef struct otm_diag {
  uint32_t flags;              /* bit k set <=> status -(k+1) happened */
  int32_t max_support;         /* largest support size of the last search */
  uint64_t n_lme_noconv, n_rm_noconv, n_inverted, n_nonfinite;
  uint64_t first_lme_noconv;   /* smallest failing MP index (UINT64_MAX: none) */
  uint64_t first_rm_noconv;
  uint64_t first_inverted;
  uint64_t first_nonfinite;    /* (a node I is reported as n_mp + I) */
  int64_t pairs_needed;        /* pair count of the last search */
  int64_t reserved[3];
} otm_diag;

/* Human-readable name of a status code (static storage). */
const char* otm_status_string(otm_status s);

/* Bytes of workspace the calls below need for these sizes (256-aligned). */
size_t otm_workspace_bytes(int64_t n_nodes, int64_t n_mp, int64_t pair_capacity);

/* Clear a device otm_diag record (enqueued on s; graph-safe, no memset). */
otm_status otm_diag_reset(otm_diag* diag, hipStream_t s);

/* Synchronise s, copy the device record into *host_out (host) and return the
 * status it encodes (the first failure kind in enum order, or OTM_OK). */
otm_status otm_diag_read(const otm_diag* diag, otm_diag* host_out, hipStream_t s);

/*
 * Support-domain search (Sec. 3 linked-cell method, Alg. 3): for every MP p
 * the nodes I with ((dx*dx + dy*dy) + dz*dz) <= r_list*r_list, dx = x_p - x_I,
 * each operation rounded on its own (no fused multiply-add), so the lists
 * are a function of the float64 inputs alone.  Nodes are binned into cells of
 * edge cell_size (>= r_list; enlarged on the device if the node bounding box
 * needs more cells than the workspace holds) and only the 27 cells around
 * each MP's cell are tested.
 *   x_nodes [3][n_nodes], x_mp [3][n_mp]: positions (device).
 *   nbr_offsets [n_mp+1], nbr_idx [pair_capacity]: output CSR (device).
 *   n_pairs_out (host): number of pairs found.
 * Synchronises s once.  Returns OTM_ERR_CAPACITY (lists not written, count in
 * *n_pairs_out) if more than pair_capacity pairs exist.
 */
otm_status otm_build_neighbors(int64_t n_nodes, const double* x_nodes, int64_t n_mp,
                               const double* x_mp, double r_list, double cell_size,
                               int64_t pair_capacity, int64_t* nbr_offsets, int32_t* nbr_idx,
                               int64_t* n_pairs_out, void* ws, size_t ws_bytes, hipStream_t s);

/*
 * LME shape functions (Sec. 2.3): N_I = Z_I / Z with
 * Z_I = exp(-beta |d_I|^2 + lambda . d_I), d_I = x_p - x_I, and lambda solving
 * sum_I N_I d_I = 0 by damped Newton from the value in lam (in/out; zero for a
 * cold start), stopping at |sum N_I d_I|_2 <= tol.  Gradients
 * dN_I = -N_I J^{-1} d_I with J = sum N_I d_I d_I^T - r r^T (the derivative of
 * the consistency condition; not printed in the paper).  Always float64
 * arithmetic; dN is written as double (OTM_FP64) or float (either mixed mode) with
 * component stride pair_capacity.  Non-convergence is recorded in diag.
 */
otm_status otm_lme_shape(int64_t n_nodes, const double* x_nodes, int64_t n_mp,
                         const double* x_mp, const int64_t* nbr_offsets, const int32_t* nbr_idx,
                         int64_t pair_capacity, double beta, double tol, int32_t max_iter,
                         double* lam, double* N, void* dN, int32_t precision, otm_diag* diag,
                         hipStream_t s);

/*
 * Start a simulation (t = 0): F = b^e = 1, epsbar = 0, T = T_r, sigma = 0,
 * lam = 0, vol left as given (initial MP volumes), du = dt * v0 (v0 [3][n_nodes]
 * device, the nodal initial velocity), then search, shape functions and the
 * first mass/force assembly, so that otm_step can follow.
 */
otm_status otm_init(otm_state* st, const otm_params* p, double dt, const double* v0,
                    int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                    hipStream_t s);

/*
 * Recompute support lists (if rebuild), shape functions and the nodal
 * mass/force for the current positions and stress (e.g. after a capacity
 * failure was fixed by a larger pair buffer).
 */
otm_status otm_refresh(otm_state* st, const otm_params* p, int32_t rebuild,
                       int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                       hipStream_t s);

/*
 * One explicit step n -> n+1 (Alg. 1, rotated so that the mass/force assembly
 * closes the step), state updated in place:
 *   nodes   du += dt^2 f / m; x* = x + du; wall projection; x = x*
 *   MPs     x_p = sum N_I x_I; dF = 1 + sum du_I (x) grad N_I; F = dF F;
 *           v = det(dF) v; constitutive update (model in p)
 *   search  if rebuild != 0 (else the lists of step n are kept; with a skin
 *           in r_list they stay valid for several steps)
 *   shapes  LME at the new MP positions (warm-started multipliers)
 *   forces  m_I = sum N_I m_p;  f_I = -sum v_p sigma_p grad N_I
 *           (- eps sum N_I e_I with params.eps_stab > 0)
 * scatter_mode selects the force assembly; the segmented mode keeps its
 * influence lists in the workspace, so pass the same workspace on every call.
 */
otm_status otm_step(otm_state* st, const otm_params* p, double dt, int32_t rebuild,
                    int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                    hipStream_t s);

/* Support lists and shape functions of one configuration (device arrays with
 * the layouts and pair capacity of the otm_state they go with). */
typedef struct otm_lists {
  int64_t* nbr_offsets;   /* [n_mp+1] */
  int32_t* nbr_idx;       /* [pair_capacity] */
  double* N;              /* [pair_capacity] */
  void* dN;               /* [3][pair_capacity], the state's precision */
} otm_lists;

/*
 * otm_step (same step, Alg. 1) with the step's support lists and shape
 * functions written into the arrays of *next instead of over the state's own.
 * The MP update reads the lists of step n from the arrays *st points to; the
 * search (rebuild != 0; with rebuild == 0 the offsets and ids of step n are
 * first copied into next) and the shape functions then fill *next, and on
 * success the four list pointers of *st are set to those of *next.  The
 * arrays *st pointed to before the call are neither written nor freed: they
 * still hold step n's lists and shape functions, so a caller that records a
 * trajectory (checkpointed adjoints) keeps them without a copy.  next's arrays
 * must not overlap the state's.  Errors as for otm_step (OTM_ERR_ARG also for
 * a NULL or misaligned next; *st is then unchanged).
 */
otm_status otm_step_into(otm_state* st, const otm_lists* next, const otm_params* p, double dt,
                         int32_t rebuild, int32_t scatter_mode, void* ws, size_t ws_bytes,
                         otm_diag* diag, hipStream_t s);

/*
 * Erosion: removes from the body the material points that met the fracture
 * criterion (Sec. 4.2, Johnson-Cook fracture separates the chip; the removal
 * of material points from the domain is the operation of the data management
 * in Sec. 3.3).  Requires params.fracture = 1 and params.eps_stab = 0.
 * Every per-MP array of *st (xp, vol, mass, lam, Fd, bed, epsbar, T, sigma,
 * failed, and qflux with conduction) is compacted in place: the surviving
 * MPs keep their order and the component stride of each [k][n_mp] array
 * becomes the new n_mp, which is written to st->n_mp; the arrays keep their
 * allocation.  failed is 0 for all survivors afterwards.
 * Node management (the same data management adds and deletes nodes; where
 * is not said): with params.insert_dist > 0, before the removal, each
 * removed MP whose support holds no node within insert_dist, and which has
 * no removed MP of smaller index within insert_dist, adds a node at its
 * position (a node at the freed surface) with its interpolated increment
 * sum_I N_Ip du_I and zero contact gap; the new nodes follow the old ones
 * in MP order, every [k][n_nodes] node array is re-strided to the new
 * st->n_nodes (room: st->node_capacity, else OTM_ERR_CAPACITY with the
 * state unchanged).  Then, as otm_refresh with rebuild = 1, the support
 * lists, shape functions and the nodal mass and force (and heat sums) of the
 * remaining body are recomputed, so that otm_step can follow.  With
 * params.delete_orphans = 1 the nodes that no support uses afterwards are
 * removed from every node array (stable order, stride st->n_nodes) and the
 * lists renumbered; otherwise such a node keeps zero mass and force.
 * *n_removed (host) receives the number of MPs removed, node_events (host,
 * 2 entries, may be NULL) the numbers of nodes added and deleted.  ws is a
 * workspace of otm_workspace_bytes(max(node_capacity, n_nodes), n_mp,
 * pair_capacity) for the state's sizes before the call.  Synchronises the
 * stream to read counts, so it cannot be captured in a graph.  Errors:
 * OTM_ERR_ARG for invalid arguments (state unchanged), OTM_ERR_CAPACITY,
 * OTM_ERR_HIP; the refresh's errors appear in diag.
 */
otm_status otm_erode(otm_state* st, const otm_params* p, int32_t scatter_mode, void* ws,
                     size_t ws_bytes, otm_diag* diag, int64_t* n_removed, int64_t* node_events,
                     hipStream_t s);

/* One stored step of a forward trajectory (host struct of device pointers,
 * float64 state as in otm_state with precision OTM_FP64).  Pair arrays N and
 * dN have component stride pair_stride.  m and f are the lumped mass and
 * force assembled for this state (the ones the next node update uses). */
typedef struct otm_tape {
  int64_t n_nodes, n_mp, pair_stride;
  const double* x;
  const double* du;
  const double* m;
  const double* f;
  const double* xp;
  const double* vol;
  const double* lam;
  const double* Fd;
  const double* bed;
  const double* epsbar;
  const double* T;
  const double* sigma;
  const int64_t* nbr_offsets;
  const int32_t* nbr_idx;
  const double* N;
  const double* dN;
} otm_tape;

/* Adjoint of a scalar loss with respect to one step's state (device,
 * float64, the layouts of otm_state; N and dN per pair of that step's lists,
 * dN with the stride of that step's tape). */
typedef struct otm_state_bar {
  double* x;
  double* du;
  double* vol;
  double* Fd;
  double* bed;
  double* epsbar;
  double* T;
  double* sigma;
  double* N;
  double* dN;
} otm_state_bar;

/* Workspace bytes of otm_step_adjoint (256-aligned). */
size_t otm_adjoint_workspace_bytes(int64_t n_nodes, int64_t n_mp);

/*
 * Reverse of one otm_step (J2 models, float64), for gradients of a loss over
 * a rollout.  tn and tn1 are the stored states before and after the step
 * (support lists frozen to theirs).  bar_next holds the adjoint of state
 * n+1 on entry and is used as scratch (its x and du receive the
 * contributions of this step before being mapped back); bar receives the
 * adjoint of state n (every field is written).  theta_bar (device, 5
 * doubles) accumulates dL/d(A, B, n, C, m) of the Johnson-Cook flow stress
 * (Sec. 4.2 hardening law) for OTM_J2_JC, or dL/d(Y0, H) in its first two
 * entries (the other three unchanged) for OTM_J2_LINEAR.  The derivative of each stage is the exact derivative of the
 * forward arithmetic: LME through the implicit function theorem on the
 * consistency condition, the return map through the spectral derivative of
 * the Hencky stress and of the exponential map and the implicit derivative
 * of the scalar return equation; wall contact and plastic onset are
 * differentiated on their active branch.  Supports longer than 48 nodes are
 * reported as OTM_ERR_SUPPORT in diag.  The stabilisation term, fracture
 * and the cutting tool have no adjoint: p->eps_stab > 0, p->fracture or
 * p->tool_enabled return OTM_ERR_ARG.
 */
otm_status otm_step_adjoint(const otm_tape* tn, const otm_tape* tn1, const otm_params* p,
                            double dt, const double* mass, otm_state_bar* bar_next,
                            otm_state_bar* bar, double* theta_bar, void* ws, size_t ws_bytes,
                            otm_diag* diag, hipStream_t s);

/*
 * Adjoint of the start of the central difference.  otm_init sets
 * du_0 = dt v0 from the nodal initial velocity v0 (the increment that starts
 * the central-difference update of the nodes, Alg. 1), and nothing else of
 * state 0 depends on v0.  Given du_bar [3][n_nodes], the adjoint of state 0's
 * du (what otm_step_adjoint wrote to bar->du for the first step of a
 * rollout), writes v0_bar [3][n_nodes] = dt du_bar: the gradient of the loss
 * with respect to every nodal initial velocity.  If dir is not NULL
 * ([3][n_nodes], a direction in the space of initial velocity fields, such
 * as the fixed field that a scalar impact speed scales), *dir_bar (device,
 * one double) receives sum_I v0_bar_I . dir_I, the loss's derivative along
 * dir, summed in a fixed order (the same bits on every run).  dir and
 * dir_bar are both NULL or both set; v0_bar must not alias du_bar or dir.
 * Enqueued on s; errors: OTM_ERR_ARG (host checks), OTM_ERR_HIP.
 */
otm_status otm_init_adjoint(int64_t n_nodes, double dt, const double* du_bar, double* v0_bar,
                            const double* dir, double* dir_bar, hipStream_t s);

/*
 * otm_step with phase markers: events[k] (host array of 7 caller-created
 * hipEvent_t; a NULL entry is skipped) are recorded on s between the phases:
 * 0 | node update | 1 | MP update | 2 | search (if rebuild) | 3, then
 *   atomic mode:      shape functions with the assembly | 4 | 6
 *   segmented mode:   influence lists (if rebuild) | 4 | shape functions with
 *                     the contribution store | 5 | ordered node sums | 6
 *   with eps_stab > 0: shape functions | 4 | assembly (atomic) | 6, or
 *                     shape functions | 4 | influence lists | 5 |
 *                     contributions and node sums (segmented) | 6.
 * Same work and results as otm_step.
 */
otm_status otm_step_profiled(otm_state* st, const otm_params* p, double dt, int32_t rebuild,
                             int32_t scatter_mode, void* ws, size_t ws_bytes, otm_diag* diag,
                             hipEvent_t* events, hipStream_t s);

/* Size of the device scratch array otm_step_noalloc uses on each device. */
#define OTM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): otm_step
 * (same step, same arguments and results) with the library's own scratch in
 * place of the caller's workspace.  The scratch is a file-scope device array
 * of OTM_STATIC_SCRATCH_BYTES (64 MiB) per device, held by each device the
 * library runs on until the process ends; the call allocates and frees
 * nothing (no hipMalloc, no library routine that allocates).
 *   Limit: states whose otm_workspace_bytes(n_nodes, n_mp, pair_capacity)
 *   exceeds OTM_STATIC_SCRATCH_BYTES are rejected with OTM_ERR_SCRATCH before
 *   anything is enqueued (about 30k MPs at 27 pairs each with the default
 *   capacity margin fit).
 *   Every call on one device shares that device's scratch, which keeps the
 *   last call's contents: nothing carries over between calls (in the
 *   segmented mode the influence lists are rebuilt from the state's support
 *   lists on every call, which costs more than otm_step with rebuild = 0).
 *   Calls that overlap in time on one device (distinct streams, or host
 *   threads) race on the scratch and give wrong results: serialise them.
 * Errors: as otm_step, plus OTM_ERR_SCRATCH; OTM_ERR_HIP if the scratch's
 * device address cannot be obtained.
 */
otm_status otm_step_noalloc(otm_state* st, const otm_params* p, double dt, int32_t rebuild,
                            int32_t scatter_mode, otm_diag* diag, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif /* OTM_H */
