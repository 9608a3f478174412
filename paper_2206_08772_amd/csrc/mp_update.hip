// Node update (central difference with lumped mass, rigid-wall projection)
// and the material-point pass: positions, incremental deformation gradient,
// F, volume and the constitutive update.
//
// Material-point pass, one workgroup per 256 MPs:
//   phase 1 (gather): groups of 16 lanes walk one MP's pairs with unit stride,
//     accumulate x_p = sum N_I x_I and H = dF - 1 = sum du_I (x) grad N_I,
//     reduce by shuffles and park the 12 sums in LDS;
//   phase 2 (update): one lane per MP reads its sums back and runs the
//     constitutive update, so the heavy scalar code uses every lane.
// The node update also writes each node as one 64-byte record
// (x, y, z, du_x, du_y, du_z, T, rate) to the workspace: the MP pass fetches
// a node with three 16-byte loads (four with conduction) and the shape
// functions its position with two, instead of one 8-byte load per value
// from the SoA arrays.
// Tensors near the identity are carried as deviations (F - 1, b^e - 1, dF - 1)
// so that their float32 forms keep relative accuracy.  The stored tensors
// have type R and the update computes in type Q: float64 / float64 in
// OTM_FP64, float32 / float32 in OTM_MIXED, float32 / float64 in
// OTM_MIXED_STORAGE.
#include <stdint.h>

#include <type_traits>

#include "constitutive.h"
#include "launch.h"
#include "otm_common.h"

namespace otm {

// ------------------------------------------------------------------- nodes
// Rigid cutting tool (Sec. 4.2 contact): a wedge rounded by the tip radius,
// extruded along z, centre of the tip circle c + t v.  The core wedge has the
// rake face along +y from c (outward normal (-1, 0)) and the flank face along
// (ca, sa) (outward normal (sa, -ca)); the gap is the signed distance to the
// core minus the tip radius.
struct ToolArgs {
  int on;
  double cx, cy, vx, vy, vz, r, sa, ca, cN, cT, mu, dt;
  const double* clock;  // [1] time of the state
  double* gt;           // [3][n] tangential gaps
};

// Contact force on node i at position xo with last increment du_old and
// lumped mass mi; updates its tangential gap.  The penalty stiffnesses are
// limited to mi / dt^2 (one step removes the whole penetration), so a light
// node does not make the explicit contact unstable; a node without mass
// feels no contact force.
OTM_DEV void tool_contact(const ToolArgs& t, int64_t n, int64_t i, const double xo[3],
                          const double du_old[3], double mi, double fc[3]) {
  const double tm = t.clock[0];
  const double dx = xo[0] - (t.cx + tm * t.vx), dy = xo[1] - (t.cy + tm * t.vy);
  const double a = -dx, b = t.sa * dx - t.ca * dy;  // n1 . d, n2 . d
  const double s1 = dy > 0.0 ? dy : 0.0;
  const double q1x = dx, q1y = dy - s1;
  const double pr2 = t.ca * dx + t.sa * dy;
  const double s2 = pr2 > 0.0 ? pr2 : 0.0;
  const double q2x = dx - s2 * t.ca, q2y = dy - s2 * t.sa;
  const double l1 = sqrt(q1x * q1x + q1y * q1y), l2 = sqrt(q2x * q2x + q2y * q2y);
  double sd, nx, ny;
  if (a <= 0.0 && b <= 0.0) {  // inside the core: nearer face
    sd = a >= b ? a : b;
    nx = a >= b ? -1.0 : t.sa;
    ny = a >= b ? 0.0 : -t.ca;
  } else {
    const bool first = l1 <= l2;
    sd = first ? l1 : l2;
    const double inv = 1.0 / (sd > 0.0 ? sd : 1.0);
    nx = (first ? q1x : q2x) * inv;
    ny = (first ? q1y : q2y) * inv;
  }
  const double g = sd - t.r;
  if (!(g < 0.0)) {
    fc[0] = fc[1] = fc[2] = 0.0;
    t.gt[i] = 0.0; t.gt[n + i] = 0.0; t.gt[2 * n + i] = 0.0;
    return;
  }
  const double nrm[3] = {nx, ny, 0.0};
  const double klim = mi > 0.0 ? mi / (t.dt * t.dt) : 0.0;
  const double kN = klim < t.cN ? klim : t.cN, kT = klim < t.cT ? klim : t.cT;
  const double tn = kN * -g;
  const double rel[3] = {du_old[0] - t.dt * t.vx, du_old[1] - t.dt * t.vy,
                         du_old[2] - t.dt * t.vz};
  const double go[3] = {t.gt[i], t.gt[n + i], t.gt[2 * n + i]};
  const double rn = rel[0] * nrm[0] + rel[1] * nrm[1] + rel[2] * nrm[2];
  const double gn = go[0] * nrm[0] + go[1] * nrm[1] + go[2] * nrm[2];
  double tt[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) tt[c] = -kT * ((go[c] - gn * nrm[c]) + (rel[c] - rn * nrm[c]));
  const double mag = sqrt(tt[0] * tt[0] + tt[1] * tt[1] + tt[2] * tt[2]);
  const double lim = t.mu * tn;
  const double scale = mag > lim ? lim / (mag > 0.0 ? mag : 1.0) : 1.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    tt[c] *= scale;
    fc[c] = tn * nrm[c] + tt[c];
    t.gt[c * n + i] = kT > 0.0 ? -tt[c] / kT : 0.0;
  }
}

__global__ void k_clock_advance(double* clock, double dt) { clock[0] += dt; }

__global__ __launch_bounds__(256) void k_node_update(int64_t n, double* __restrict__ x,
                                                     double* __restrict__ du,
                                                     double* __restrict__ m,
                                                     double* __restrict__ f, double dt2,
                                                     int wall, double wx0, double wx1,
                                                     double wx2, double wn0, double wn1,
                                                     double wn2, int zero_mf,
                                                     double4* __restrict__ packed,
                                                     int64_t n_mp, otm_diag* diag,
                                                     ToolArgs tool, double* __restrict__ heat,
                                                     double cp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double mi = m[i];
  // conduction: the nodal temperature h_I / m_I and its rate Q_I / (Cp m_I)
  // from the sums of the last assembly (0 at a node without mass)
  double Ti = 0.0, Ri = 0.0;
  if (heat != nullptr && mi > 0.0) {
    Ti = heat[i] / mi;
    Ri = heat[n + i] / (cp * mi);
  }
  double u[3], xs[3], xo[3], fi[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    xo[c] = x[c * n + i];
    u[c] = du[c * n + i];
    fi[c] = f[c * n + i];
  }
  if (tool.on) {
    double fc[3];
    tool_contact(tool, n, i, xo, u, mi, fc);
#pragma unroll
    for (int c = 0; c < 3; ++c) fi[c] += fc[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    // a node outside every support (no mass, no force) keeps its increment
    u[c] = u[c] + (mi > 0.0 ? dt2 * fi[c] / mi : 0.0);
    xs[c] = xo[c] + u[c];
  }
  if (wall) {
    const double g = (xs[0] - wx0) * wn0 + (xs[1] - wx1) * wn1 + (xs[2] - wx2) * wn2;
    if (g < 0.0) {
      xs[0] -= g * wn0; xs[1] -= g * wn1; xs[2] -= g * wn2;
#pragma unroll
      for (int c = 0; c < 3; ++c) u[c] = xs[c] - xo[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    x[c * n + i] = xs[c];
    du[c * n + i] = u[c];
  }
  if (!(isfinite(xs[0]) && isfinite(xs[1]) && isfinite(xs[2])))
    diag_fail(diag, OTM_ERR_NONFINITE, (uint64_t)(n_mp + i));
  if (zero_mf) {
    m[i] = 0.0;
    f[i] = 0.0; f[n + i] = 0.0; f[2 * n + i] = 0.0;
    if (heat != nullptr) { heat[i] = 0.0; heat[n + i] = 0.0; }
  }
  packed[2 * i] = make_double4(xs[0], xs[1], xs[2], u[0]);
  packed[2 * i + 1] = make_double4(u[1], u[2], Ti, Ri);
}

__global__ __launch_bounds__(256) void k_pack_nodes(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ du,
                                                    double4* __restrict__ packed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  packed[2 * i] = make_double4(x[i], x[n + i], x[2 * n + i], du[i]);
  packed[2 * i + 1] = make_double4(du[n + i], du[2 * n + i], 0.0, 0.0);
}

void launch_pack_nodes(const otm_state& st, double4* packed, hipStream_t s) {
  const int64_t n = st.n_nodes;
  if (n <= 0) return;
  k_pack_nodes<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, st.x, st.du, packed);
}

void launch_node_update(const otm_state& st, const otm_params& p, double dt, bool zero_mf,
                        double4* packed, otm_diag* diag, hipStream_t s) {
  const int64_t n = st.n_nodes;
  if (n <= 0) return;
  ToolArgs t{};
  if (p.tool_enabled) {
    t.on = 1;
    t.cx = p.tool_c[0]; t.cy = p.tool_c[1];
    t.vx = p.tool_v[0]; t.vy = p.tool_v[1]; t.vz = p.tool_v[2];
    t.r = p.tool_r;
    t.sa = std::sin(p.tool_clearance);
    t.ca = std::cos(p.tool_clearance);
    t.cN = p.tool_cN; t.cT = p.tool_cT; t.mu = p.tool_mu;
    t.dt = dt;
    t.clock = st.clock;
    t.gt = st.tool_gt;
  }
  k_node_update<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(
      n, st.x, st.du, st.m, st.f, dt * dt, p.wall_enabled, p.wall_x[0], p.wall_x[1],
      p.wall_x[2], p.wall_n[0], p.wall_n[1], p.wall_n[2], zero_mf ? 1 : 0, packed, st.n_mp,
      diag, t, p.kappa > 0.0 ? st.heat : nullptr, p.Cp);
}

// ----------------------------------------------------- material-point pass
constexpr int kMpBlock = 256;
constexpr int kGather = 16;            // lanes per MP in the gather phase
constexpr int kSlots = 32 / kGather;   // pairs per lane loaded branch-free

// Conduction (COND): the gather also sums grad T_p = sum_I T_I grad N_Ip and
// sum_I N_Ip rate_I from the node records' (T_I, rate_I), kept in sums[13..16]
// (past the slots that phase 2 parks values in); phase 2 adds
// dt sum N rate to T_{n+1} and stores the flux -kappa grad T_p.
//
// PAIRED: a lane's two slots are two consecutive pairs starting at an even
// index, so idx, N and each component of grad N come in one load of two
// values (8 or 16 bytes) instead of two; this needs idx 8-byte, N and grad N
// 2 sizeof(R)-byte aligned and an even capacity (the launcher checks).
template <typename R, bool COND, typename Q = R, bool PAIRED = false>
__global__ __launch_bounds__(kMpBlock) void k_mp_update(
    const double4* __restrict__ nodes, int64_t n_nodes, int64_t n_mp,
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ idx,
    int64_t cap, const double* __restrict__ N, const R* __restrict__ dN,
    double* __restrict__ xp, double* __restrict__ vol, R* __restrict__ Fd, R* __restrict__ bed,
    double* __restrict__ epsbar, double* __restrict__ T, R* __restrict__ sigma, Mat<Q> M,
    double* __restrict__ xp_prev, double* __restrict__ dFm1, int32_t* __restrict__ failed,
    double* __restrict__ clock, double dt, otm_diag* diag, double kappa,
    double* __restrict__ qflux) {
  // phase 1: the 12 (16 with conduction) gathered sums of each MP; phase 2:
  // the MP's eigenvectors, logarithmic strains and J parked in sums[0..12]
  // over the return-map solve (each lane only touches its own column)
  constexpr int kSums = COND ? 17 : 13;
  constexpr int kGathered = COND ? 16 : 12;
  // rows padded by one double, so that the lanes of a group writing the
  // sums of one MP hit different LDS banks
  __shared__ double sums[kSums][kMpBlock + 1];
  __shared__ int64_t row[kMpBlock + 1];
  const int64_t base = (int64_t)xcd_block() * kMpBlock;
  const int tid = threadIdx.x;
  // the tool's clock moves on here: the node update before has read it and
  // the next one comes after this kernel
  if (clock != nullptr && blockIdx.x == 0 && tid == 0) clock[0] += dt;
  const bool lists_ok = offsets[n_mp] <= cap;
  const bool have_nodes = n_nodes > 0 && cap > 0;
  // the block's row offsets, read once (rows past the end are empty)
  for (int i = tid; i <= kMpBlock; i += kMpBlock) row[i] = offsets[min(base + i, n_mp)];
  __syncthreads();

  // phase 1: gather with kGather lanes per MP in kGather rounds of
  // kMpBlock / kGather MPs, software-pipelined three deep.  Round r issues the
  // node gathers of round r + 1, then sums round r, then issues the pair data
  // (N, grad N) of round r + 2 and the node ids of round r + 3.  Vector loads
  // complete in issue order, so a wait can only leave younger loads in flight;
  // with this order every wait is for pair data issued two rounds earlier or
  // for gathers issued one round earlier, never for the newest HBM loads.
  // Register sets alternate with the parity of the round.  Slot k of lane l
  // is pair k * kGather + l of the row, or with PAIRED pair q0 + k, q0 = the
  // row's start rounded down to even + 2 l (a slot before the start or past
  // the end is unused).  Unused slots get weight 0 and gather node 0; their
  // pair data is pair 0's (or, with PAIRED, the neighbouring pair loaded
  // with a used one), so all loads are branch-free.  The pairs past the
  // slots (long rows) are added after the pipeline.
  if (lists_ok && have_nodes) {
    const int lane = tid % kGather;
    const int grp = tid / kGather;
    constexpr int kPer = kMpBlock / kGather;
    struct Ids { int32_t i[kSlots]; bool use[kSlots]; };
    // grad N stays in its stored type until it is used, so that no
    // conversion has to wait for a load in the round that issues it
    struct Pairs { double w[kSlots]; R g0[kSlots], g1[kSlots], g2[kSlots]; };
    // a node record as three 16-byte pieces: (x, y), (z, du_x), (du_y, du_z),
    // and with conduction a fourth, (T_I, rate_I)
    struct Nodes {
      double2 a[kSlots], b[kSlots], c[kSlots], d[COND ? kSlots : 1];
      bool use[kSlots];
    };
    const double2* __restrict__ nd2 = reinterpret_cast<const double2*>(nodes);
    auto slot = [&](int r, int k, bool& use) {
      const int local = r * kPer + grp;
      const int64_t q = row[local] + k * kGather + lane;
      use = q < row[local + 1];
      return use ? q : (int64_t)0;
    };
    // PAIRED: the lane's first pair (even; q0 + 1 < capacity whenever
    // q0 < capacity, the capacity being even), or 0 if neither slot is used
    static_assert(!PAIRED || kSlots == 2, "two consecutive pairs per lane");
    auto pair0 = [&](int r, bool (&use)[kSlots]) {
      const int local = r * kPer + grp;
      const int64_t a = row[local], b = row[local + 1];
      const int64_t q0 = (a & ~(int64_t)1) + 2 * lane;
      use[0] = q0 >= a && q0 < b;
      use[1] = q0 + 1 < b;
      return use[0] || use[1] ? q0 : (int64_t)0;
    };
    using R2 = std::conditional_t<std::is_same_v<R, double>, double2, float2>;
    auto load_ids = [&](Ids& s, int r) {
      if constexpr (PAIRED) {
        const int2 v = *reinterpret_cast<const int2*>(idx + pair0(r, s.use));
        s.i[0] = v.x;
        s.i[1] = v.y;
      } else {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) s.i[k] = idx[slot(r, k, s.use[k])];
      }
    };
    auto load_pairs = [&](Pairs& s, int r) {
      if constexpr (PAIRED) {
        bool use[kSlots];
        const int64_t q0 = pair0(r, use);
        const double2 w = *reinterpret_cast<const double2*>(N + q0);
        const R2 g0 = *reinterpret_cast<const R2*>(dN + q0);
        const R2 g1 = *reinterpret_cast<const R2*>(dN + cap + q0);
        const R2 g2 = *reinterpret_cast<const R2*>(dN + 2 * cap + q0);
        s.w[0] = w.x; s.w[1] = w.y;
        s.g0[0] = g0.x; s.g0[1] = g0.y;
        s.g1[0] = g1.x; s.g1[1] = g1.y;
        s.g2[0] = g2.x; s.g2[1] = g2.y;
      } else {
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
          bool use;
          const int64_t q = slot(r, k, use);
          s.w[k] = N[q];
          s.g0[k] = dN[q];
          s.g1[k] = dN[cap + q];
          s.g2[k] = dN[2 * cap + q];
        }
      }
    };
    auto load_nodes = [&](Nodes& s, const Ids& ids) {
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        const int32_t I = ids.use[k] ? ids.i[k] : 0;  // idx[0] is unset without pairs
        s.use[k] = ids.use[k];
        s.a[k] = nd2[4 * (int64_t)I];
        s.b[k] = nd2[4 * (int64_t)I + 1];
        s.c[k] = nd2[4 * (int64_t)I + 2];
        if constexpr (COND) s.d[k] = nd2[4 * (int64_t)I + 3];
      }
    };
    auto sum_round = [&](int r, const Nodes& nd, const Pairs& pr) {
      double a[kGathered] = {};
#pragma unroll
      for (int k = 0; k < kSlots; ++k) {
        const double wt = nd.use[k] ? pr.w[k] : 0.0;
        const double h0 = nd.use[k] ? (double)pr.g0[k] : 0.0;
        const double h1 = nd.use[k] ? (double)pr.g1[k] : 0.0;
        const double h2 = nd.use[k] ? (double)pr.g2[k] : 0.0;
        const double x0 = nd.a[k].x, x1 = nd.a[k].y, x2 = nd.b[k].x;
        const double u0 = nd.b[k].y, u1 = nd.c[k].x, u2 = nd.c[k].y;
        a[0] += wt * x0; a[1] += wt * x1; a[2] += wt * x2;
        a[3] += u0 * h0; a[4] += u0 * h1; a[5] += u0 * h2;
        a[6] += u1 * h0; a[7] += u1 * h1; a[8] += u1 * h2;
        a[9] += u2 * h0; a[10] += u2 * h1; a[11] += u2 * h2;
        if constexpr (COND) {
          const double tI = nd.d[k].x, rI = nd.d[k].y;
          a[12] += tI * h0; a[13] += tI * h1; a[14] += tI * h2;
          a[15] += wt * rI;
        }
      }
      // each of the group's lanes ends with the total of one sum (or none)
      // and writes it: one store instead of kGathered from one lane
      int c;
      const double t = row_sum_scatter<kGathered>(a, c);
      if (c >= 0) sums[COND && c >= 12 ? c + 1 : c][r * kPer + grp] = t;
    };
    Ids i0, i1;
    Pairs p0, p1;
    Nodes n0, n1;
    // the prologue issues in the loop's own order (pairs r, ids r + 1,
    // gathers r, pairs r + 1, ids r + 2), so the waits at the loop head need
    // not assume an older order
    load_ids(i0, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_pairs(p0, 0);
    __builtin_amdgcn_sched_barrier(0);
    load_ids(i1, 1);
    __builtin_amdgcn_sched_barrier(0);
    load_nodes(n0, i0);
    __builtin_amdgcn_sched_barrier(0);
    load_pairs(p1, 1);
    __builtin_amdgcn_sched_barrier(0);
    load_ids(i0, 2);
    static_assert(kGather % 2 == 0 && kGather >= 6, "rounds are taken in pairs");
    // rounds r, r + 1, fetching ahead up to round r + 4 (with_ids: the ids of
    // round r + 4 exist)
    auto two_rounds = [&](int r, bool with_ids) {
      __builtin_amdgcn_sched_barrier(0);
      load_nodes(n1, i1);             // gathers of round r + 1
      __builtin_amdgcn_sched_barrier(0);
      sum_round(r, n0, p0);
      __builtin_amdgcn_sched_barrier(0);
      load_pairs(p0, r + 2);
      load_ids(i1, r + 3);
      __builtin_amdgcn_sched_barrier(0);
      load_nodes(n0, i0);             // gathers of round r + 2
      __builtin_amdgcn_sched_barrier(0);
      sum_round(r + 1, n1, p1);
      __builtin_amdgcn_sched_barrier(0);
      load_pairs(p1, r + 3);
      if (with_ids) load_ids(i0, r + 4);
    };
    for (int r = 0; r < kGather - 4; r += 2) two_rounds(r, true);
    two_rounds(kGather - 4, false);
    // the last two rounds: nothing left to fetch ahead
    __builtin_amdgcn_sched_barrier(0);
    load_nodes(n1, i1);
    __builtin_amdgcn_sched_barrier(0);
    sum_round(kGather - 2, n0, p0);
    __builtin_amdgcn_sched_barrier(0);
    sum_round(kGather - 1, n1, p1);
    __builtin_amdgcn_sched_barrier(0);
    // long rows: the pairs past the slots, summed per group and added to the
    // row's sums by the group's lane 0; the round totals were written by
    // other lanes of the same wave, so a wave-level fence comes first
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int r = 0; r < kGather; ++r) {
      const int local = r * kPer + grp;
      const int64_t o0 = row[local], o1 = row[local + 1];
      const int64_t done = (PAIRED ? (o0 & ~(int64_t)1) : o0) + kSlots * kGather;
      if (o1 <= done) continue;  // uniform within the group
      double a[kGathered] = {};
      for (int64_t q = done + lane; q < o1; q += kGather) {
        const int32_t J = idx[q];
        const double wt = N[q];
        const double h0 = (double)dN[q], h1 = (double)dN[cap + q], h2 = (double)dN[2 * cap + q];
        const double2 ra = nd2[4 * (int64_t)J], rb = nd2[4 * (int64_t)J + 1];
        const double2 rc = nd2[4 * (int64_t)J + 2];
        a[0] += wt * ra.x; a[1] += wt * ra.y; a[2] += wt * rb.x;
        a[3] += rb.y * h0; a[4] += rb.y * h1; a[5] += rb.y * h2;
        a[6] += rc.x * h0; a[7] += rc.x * h1; a[8] += rc.x * h2;
        a[9] += rc.y * h0; a[10] += rc.y * h1; a[11] += rc.y * h2;
        if constexpr (COND) {
          const double2 rd = nd2[4 * (int64_t)J + 3];
          a[12] += rd.x * h0; a[13] += rd.x * h1; a[14] += rd.x * h2;
          a[15] += wt * rd.y;
        }
      }
#pragma unroll
      for (int c = 0; c < kGathered; ++c) a[c] = group_sum<kGather>(a[c]);
      if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) sums[c][local] += a[c];
        if constexpr (COND) {
#pragma unroll
          for (int c = 12; c < 16; ++c) sums[c + 1][local] += a[c];
        }
      }
    }
  } else {
    for (int i = tid; i < kSums * kMpBlock; i += kMpBlock) sums[i / kMpBlock][i % kMpBlock] = 0.0;
  }
  // phase 2's inputs of this lane's MP, requested before the barrier: their
  // latency overlaps the end of the gathers and the update waits for them
  // once instead of once per input as it reaches it
  const int64_t p = base + tid;
  const bool mine = p < n_mp && lists_ok;
  double vol_n = 0.0, ebn = 0.0, Tn = 0.0;
  R fd_n[9], bd_n[6];
  if (mine) {
    vol_n = vol[p];
#pragma unroll
    for (int k = 0; k < 9; ++k) fd_n[k] = Fd[k * n_mp + p];
#pragma unroll
    for (int k = 0; k < 6; ++k) bd_n[k] = bed[k * n_mp + p];
    ebn = epsbar[p];
    Tn = T[p];
  }
  __syncthreads();

  // phase 2: one lane per MP
  if (!mine) return;
  M3<double> H;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) H.a[i][j] = sums[3 + 3 * i + j][tid];
  const double xnew[3] = {sums[0][tid], sums[1][tid], sums[2][tid]};
  bool finite = isfinite(xnew[0]) && isfinite(xnew[1]) && isfinite(xnew[2]);
  // conduction: this step's increment and the new flux (with step n's
  // shape functions and the nodal field of the node update)
  double dTc = 0.0;
  if constexpr (COND) {
    dTc = dt * sums[16][tid];
#pragma unroll
    for (int c = 0; c < 3; ++c) qflux[c * n_mp + p] = -kappa * sums[13 + c][tid];
  }
  const double detdF = 1.0 + det_one_plus_minus_one(H);
  // a failed MP (fracture) carries nothing, so its inversion does not matter
  // (loaded here: a value merged over the null-pointer branch would be
  // waited for before the barrier; here this one wait covers all the above)
  const bool was_failed = failed != nullptr && failed[p] != 0;
  if (!(detdF > 0.0) && !was_failed) diag_fail(diag, OTM_ERR_INVERTED, (uint64_t)p);
  vol[p] = detdF * vol_n;
  if (dFm1 != nullptr) {  // history of the stabilisation term
#pragma unroll
    for (int c = 0; c < 3; ++c) xp_prev[c * n_mp + p] = xp[c * n_mp + p];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) dFm1[(3 * i + j) * n_mp + p] = H.a[i][j];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) xp[c * n_mp + p] = xnew[c];

  // F - 1 <- H + Fd + H Fd
  M3<Q> h, fo, fn;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      h.a[i][j] = (Q)H.a[i][j];
      fo.a[i][j] = fd_n[3 * i + j];
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      fn.a[i][j] = h.a[i][j] + fo.a[i][j] +
                   (h.a[i][0] * fo.a[0][j] + h.a[i][1] * fo.a[1][j] + h.a[i][2] * fo.a[2][j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Fd[(3 * i + j) * n_mp + p] = fn.a[i][j];
  const Q Jm1 = det_one_plus_minus_one(fn);
  Q J = Q(1) + Jm1;

  S3<Q> sig;
  if (M.model == OTM_NEOHOOKE) {
    // sigma = (mu/J)(b - 1) + (lambda ln J / J) 1, b - 1 = X + X^T + X X^T
    const int ii[6] = {0, 1, 2, 0, 1, 0}, jj[6] = {0, 1, 2, 1, 2, 2};
    const Q lnJ = m_log1p(Jm1);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int i = ii[c], j = jj[c];
      const Q bm1 = fn.a[i][j] + fn.a[j][i] +
                    (fn.a[i][0] * fn.a[j][0] + fn.a[i][1] * fn.a[j][1] + fn.a[i][2] * fn.a[j][2]);
      sig.v[c] = M.mu / J * bm1 + (c < 3 ? M.lamL * lnJ / J : Q(0));
    }
  } else if (was_failed) {
    // eroded: no stress; b^e, epsbar and T stay as they were (but for the
    // conduction increment: a failed MP still holds heat)
#pragma unroll
    for (int c = 0; c < 6; ++c) sig.v[c] = Q(0);
    if constexpr (COND) T[p] = Tn + dTc;
  } else {
    // trial elastic left Cauchy-Green tensor, as a deviation from 1:
    // b_tr - 1 = H + H^T + H H^T + (1+H) Bd (1+H)^T
    S3<Q> bd;
#pragma unroll
    for (int c = 0; c < 6; ++c) bd.v[c] = bd_n[c];
    const M3<Q> B = full(bd);
    M3<Q> HB;  // (1 + H) Bd
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        HB.a[i][j] = B.a[i][j] + h.a[i][0] * B.a[0][j] + h.a[i][1] * B.a[1][j] + h.a[i][2] * B.a[2][j];
    S3<Q> dtr;
    const int ii[6] = {0, 1, 2, 0, 1, 0}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int i = ii[c], j = jj[c];
      // (1+H) Bd (1+H)^T = HB + HB H^T
      const Q hbh = HB.a[i][j] + HB.a[i][0] * h.a[j][0] + HB.a[i][1] * h.a[j][1] + HB.a[i][2] * h.a[j][2];
      dtr.v[c] = h.a[i][j] + h.a[j][i] +
                 (h.a[i][0] * h.a[j][0] + h.a[i][1] * h.a[j][1] + h.a[i][2] * h.a[j][2]) + hbh;
    }
    Q d[3], V[3][3];
    jacobi_eig(dtr, d, V);
    Q e[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) e[a] = Q(0.5) * m_log1p(d[a]);
    Q tr = e[0] + e[1] + e[2];
    Q dev[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) dev[a] = e[a] - tr / Q(3);
    const Q q_tr = Q(2) * M.mu * m_sqrt(Q(1.5) * (dev[0] * dev[0] + dev[1] * dev[1] + dev[2] * dev[2]));
    Q Ts = Q(0);
    if (M.model == OTM_J2_JC) {
      Q t = (Q)((Tn - (double)M.Tr) / ((double)M.Tm - (double)M.Tr));
      Ts = t < Q(0) ? Q(0) : (t > Q(1) ? Q(1) : t);
    }
    Q sy0, dsy0;
    flow_stress(M, (Q)ebn, Q(0), Ts, sy0, dsy0);
    Q deps = Q(0), c = Q(0);
    if (q_tr > sy0) {
      // the solve is the register peak of the kernel: park what it does not
      // use in LDS and read it back afterwards
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) sums[3 * i + j][tid] = (double)V[i][j];
        sums[9 + i][tid] = (double)e[i];
      }
      sums[12][tid] = (double)J;
      bool ok;
      deps = solve_return(M, q_tr, (Q)ebn, Ts, sy0, ok);
      if (!ok) diag_fail(diag, OTM_ERR_RM_NOCONV, (uint64_t)p);
      c = Q(3) * M.mu * deps / q_tr;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) V[i][j] = (Q)sums[3 * i + j][tid];
        e[i] = (Q)sums[9 + i][tid];
      }
      J = (Q)sums[12][tid];
      tr = e[0] + e[1] + e[2];
#pragma unroll
      for (int a = 0; a < 3; ++a) dev[a] = e[a] - tr / Q(3);
    }
    Q bnew[3], tau[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const Q ea = e[a] - c * dev[a];
      bnew[a] = m_expm1(Q(2) * ea);
      tau[a] = (M.K * tr + Q(2) * M.mu * (Q(1) - c) * dev[a]) / J;
    }
    const S3<Q> bn = spectral_compose(V, bnew);
    sig = spectral_compose(V, tau);
#pragma unroll
    for (int k = 0; k < 6; ++k) bed[k * n_mp + p] = bn.v[k];
    const double eb_new = ebn + (double)deps;
    epsbar[p] = eb_new;
    double T_new = Tn;
    if (M.model == OTM_J2_JC) {
      T_new = (Tn + dTc) + (double)(M.chi * (Q(1) - c) * q_tr * deps / M.rhoCp);
      T[p] = T_new;
    }
    if (failed != nullptr && eb_new > 0.0) {
      // Johnson-Cook fracture criterion (Sec. 4.2) on the principal Cauchy
      // stresses: triaxiality = mean / von Mises stress
      const double s0 = tau[0], s1 = tau[1], s2 = tau[2];
      const double sm = (s0 + s1 + s2) / 3.0;
      const double e0 = s0 - sm, e1 = s1 - sm, e2 = s2 - sm;
      const double sv = sqrt(1.5 * (e0 * e0 + e1 * e1 + e2 * e2));
      const double eta = sv > 0.0 ? sm / sv : 0.0;
      const double ratio = (double)deps / M.rate0dt_d;
      const double lr = ratio > 1.0 ? log(ratio) : 0.0;
      double ts = (T_new - (double)M.Tr) / ((double)M.Tm - (double)M.Tr);
      ts = ts < 0.0 ? 0.0 : (ts > 1.0 ? 1.0 : ts);
      const double ef = (M.jd[0] + M.jd[1] * exp(M.jd[2] * eta)) * (1.0 + M.jd[3] * lr) *
                        (1.0 + M.jd[4] * ts);
      if (eb_new >= ef) {
        failed[p] = 1;
#pragma unroll
        for (int k = 0; k < 6; ++k) sig.v[k] = Q(0);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    sigma[k * n_mp + p] = sig.v[k];
    finite = finite && isfinite((double)sig.v[k]);
  }
  if (!finite) diag_fail(diag, OTM_ERR_NONFINITE, (uint64_t)p);
}

void launch_mp_update(const otm_state& st, const otm_params& p, double dt,
                      const double4* packed, otm_diag* diag, hipStream_t s) {
  const int64_t n = st.n_mp;
  if (n <= 0) {
    if (p.tool_enabled) k_clock_advance<<<1, 1, 0, s>>>(st.clock, dt);
    return;
  }
  const unsigned nb = (unsigned)((n + kMpBlock - 1) / kMpBlock);
  double* hist_x = p.eps_stab > 0.0 ? st.xp_prev : nullptr;
  double* hist_f = p.eps_stab > 0.0 ? st.dFm1 : nullptr;
  int32_t* frac = p.fracture ? st.failed : nullptr;
  double* clock = p.tool_enabled ? st.clock : nullptr;
  auto run = [&](auto kernel, auto* dn, auto* fd, auto* bd, auto* sg, auto mat) {
    kernel<<<nb, kMpBlock, 0, s>>>(packed, st.n_nodes, n, st.nbr_offsets, st.nbr_idx,
                                   st.pair_capacity, st.N, dn, st.xp, st.vol, fd, bd, st.epsbar,
                                   st.T, sg, mat, hist_x, hist_f, frac, clock, dt, diag, p.kappa,
                                   st.qflux);
  };
  // paired pair loads where the arrays allow them (see k_mp_update)
  const size_t dn_size = st.precision == OTM_FP64 ? sizeof(double) : sizeof(float);
  const bool paired = st.pair_capacity % 2 == 0 && (uintptr_t)st.nbr_idx % 8 == 0 &&
                      (uintptr_t)st.N % 16 == 0 && (uintptr_t)st.dN % (2 * dn_size) == 0;
  const bool cond = p.kappa > 0.0;
  auto pick = [&](auto r_tag, auto q_tag, auto dn, auto fd, auto bd, auto sg, auto m) {
    using R = decltype(r_tag);
    using Q = decltype(q_tag);
    if (cond) {
      if (paired) run(k_mp_update<R, true, Q, true>, dn, fd, bd, sg, m);
      else run(k_mp_update<R, true, Q, false>, dn, fd, bd, sg, m);
    } else {
      if (paired) run(k_mp_update<R, false, Q, true>, dn, fd, bd, sg, m);
      else run(k_mp_update<R, false, Q, false>, dn, fd, bd, sg, m);
    }
  };
  if (st.precision == OTM_FP64) {
    pick(double{}, double{}, (const double*)st.dN, (double*)st.Fd, (double*)st.bed,
         (double*)st.sigma, make_mat<double>(p, dt));
    return;
  }
  float *fd = (float*)st.Fd, *bd = (float*)st.bed, *sg = (float*)st.sigma;
  const float* dn = (const float*)st.dN;
  if (st.precision == OTM_MIXED)  // the return map in float32
    pick(float{}, float{}, dn, fd, bd, sg, make_mat<float>(p, dt));
  else  // float32 storage, float64 arithmetic
    pick(float{}, double{}, dn, fd, bd, sg, make_mat<double>(p, dt));
}

// ------------------------------------------------------------------- t = 0
template <typename R>
__global__ void k_init_mp(int64_t n, R* Fd, R* bed, R* sigma, double* epsbar, double* T,
                          double* lam, double Tr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  for (int c = 0; c < 9; ++c) Fd[c * n + p] = R(0);
  for (int c = 0; c < 6; ++c) { bed[c * n + p] = R(0); sigma[c * n + p] = R(0); }
  epsbar[p] = 0.0;
  T[p] = Tr;
  lam[p] = 0.0; lam[n + p] = 0.0; lam[2 * n + p] = 0.0;
}

__global__ void k_init_nodes(int64_t n, double* du, const double* v0, double dt, double* gt,
                             double* clock) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && clock != nullptr) clock[0] = 0.0;
  if (i >= n) return;
  for (int c = 0; c < 3; ++c) du[c * n + i] = dt * v0[c * n + i];
  if (gt != nullptr)
    for (int c = 0; c < 3; ++c) gt[c * n + i] = 0.0;
}

__global__ void k_init_failed(int64_t n, int32_t* failed) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) failed[p] = 0;
}

void launch_init_fields(const otm_state& st, const otm_params& p, double dt, const double* v0,
                        hipStream_t s) {
  if (st.n_mp > 0) {
    const unsigned nb = (unsigned)((st.n_mp + 255) / 256);
    if (st.precision == OTM_FP64)
      k_init_mp<double><<<nb, 256, 0, s>>>(st.n_mp, (double*)st.Fd, (double*)st.bed,
                                           (double*)st.sigma, st.epsbar, st.T, st.lam, p.T_r);
    else
      k_init_mp<float><<<nb, 256, 0, s>>>(st.n_mp, (float*)st.Fd, (float*)st.bed,
                                          (float*)st.sigma, st.epsbar, st.T, st.lam, p.T_r);
  }
  if (p.fracture && st.n_mp > 0)
    k_init_failed<<<(unsigned)((st.n_mp + 255) / 256), 256, 0, s>>>(st.n_mp, st.failed);
  if (p.kappa > 0.0 && st.n_mp > 0) launch_zero(st.qflux, 3 * st.n_mp, s);  // no flux at t = 0
  double* gt = p.tool_enabled ? st.tool_gt : nullptr;
  double* clock = p.tool_enabled ? st.clock : nullptr;
  if (st.n_nodes > 0 || clock != nullptr) {  // one workgroup at least: it sets the clock
    const unsigned nb = st.n_nodes > 0 ? (unsigned)((st.n_nodes + 255) / 256) : 1u;
    k_init_nodes<<<nb, 256, 0, s>>>(st.n_nodes, st.du, v0, dt, gt, clock);
  }
}

}  // namespace otm
