// mppi_dev.hpp -- device-resident data layouts shared by the host runtime and
// the HIP kernels of the MPPI hot path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mppi {

constexpr int kMaxBodies = 64;
constexpr int kMaxContacts = 32;
constexpr int kMaxChildren = 8;
constexpr int kMaxKnots = 64;
constexpr int kMaxChains = 8;    // chain schedule: kinematic chains (lanes) per rollout
constexpr int kMaxLevels = 16;   // chain schedule: tree depth + 1
constexpr int kRow = 68;         // floats per body row of the chain schedule's table
constexpr int kCt = 8;           // floats per contact row of that table

// Body row of the chain schedule's table (floats; integer fields stored as bits):
//   [0,27) P   [27,30) p_tree   [30,33) axis_p   [33,36) com   [36,42) Ic   42 mass
//   43 kp  44 kd  45 tau_max  46 armature  47 q0 (running-cost posture, per instance)
//   48 parent  49 c_begin  50 c_count  51 n_child  52 heavy child (same chain) or -1
//   53 attach slot written by this body or -1  54 chain  55 depth  [56,64) children
// Contact row: [0,3) position in the body frame, 3 f0z (per instance), 4 original index.
namespace row {
enum : int { P = 0, p_tree = 27, axis_p = 30, com = 33, Ic = 36, mass = 42, kp = 43, kd = 44, taumax = 45, arm = 46,
             q0 = 47, parent = 48, c_begin = 49, c_count = 50, n_child = 51, heavy = 52, att = 53, chain = 54,
             depth = 55, child = 56 };
}

// Team schedule records are indexed by slot: the bodies numbered by (depth,
// chain), so the bodies one level works on sit in consecutive slots.  Per slot and coordinate
// lane k the constants of its joint take 16 floats (stride kTeamK): rows k of P0,
// P1, P2 with columns in rotated order (entry i = column k + i), then p_tree and
// axis_p in the same order (components k, k+1, k+2), then [15] = the joint's
// armature (k = 0) or the bit mask of the chains whose first body hangs off
// this body (k = 1, as integer bits).  The strides (20 floats per lane, 60 per
// slot; 8 and 28 for the frame records) put the three lanes of a team and the
// teams of two neighbouring chains on different LDS banks.
constexpr int kTeamK = 20;
constexpr int kTeamSlot = 60;
constexpr int kTeamRow = 3 * 16;   // host copy per body
constexpr int kFrSlot = 28;

// Kinematic tree in the layout the rollout lanes read: one entry per body,
// contacts sorted by body.  Precomputed on the host from mppi_model_desc:
//  * the joint rotation C(q) = R_tree Rot(axis, q) is stored as
//    C = P0 + cos(q) P1 + sin(q) P2 (Rodrigues' formula distributed over R_tree);
//  * axis_p = R_tree axis, the joint axis in the parent frame.
struct DevModel {
  int32_t nb, fb, nu, nc, nsub, ee_body, n_levels, max_depth;
  float k, d, mu, eps, g, mtot;
  float ee_pos[3];
  int32_t parent[kMaxBodies];
  int32_t depth[kMaxBodies];
  int32_t n_child[kMaxBodies];
  int32_t child[kMaxBodies][kMaxChildren];
  int32_t c_begin[kMaxBodies];
  int32_t c_count[kMaxBodies];
  float P[kMaxBodies][27];  // P0 | P1 | P2, row-major 3x3 each
  float axis_p[kMaxBodies][3];
  float p_tree[kMaxBodies][3];
  float mass[kMaxBodies];
  float com[kMaxBodies][3];
  float Ic[kMaxBodies][6];  // xx yy zz xy xz yz about the com, body frame
  float qmin[kMaxBodies], qmax[kMaxBodies], taumax[kMaxBodies], kp[kMaxBodies], kd[kMaxBodies];
  float arm[kMaxBodies];    // reflected rotor inertia per joint
  float cpos[kMaxContacts][3];  // sorted by body
  int32_t corig[kMaxContacts];  // original contact index
  // Chain schedule: heavy-path decomposition of the tree into chains (a body
  // continues the chain of its parent when it heads the parent's largest
  // subtree).  A chain hangs off another chain's body through an attach slot.
  int32_t chain_ok;                             // 1 if the tree fits the chain schedule
  int32_t n_chains, chain_lanes, n_att;
  int32_t chain_body[kMaxChains][kMaxLevels];   // body of chain c at depth d, or -1
  int32_t chain_first[kMaxChains];              // depth of the chain's first body
  int32_t chain_att[kMaxChains];                // attach slot its first body reads, or -1 (a root)
  alignas(16) float rows[kMaxBodies][kRow];     // body rows (layout above), read as float4
  float ctab[kMaxContacts][kCt];                // contact rows
  // Team schedule: the chains above, each on a block of team_block lanes
  // (team_lanes per rollout); per body and coordinate lane k the constants of
  // its joint in rotated order (see team_table_floats).
  int32_t team_ok, team_block, team_lanes, team_slots;
  int32_t chain_len[kMaxChains];                // bodies of chain c
  int32_t chain_parent[kMaxChains];             // parent body of its first body, or -1
  int32_t team_slot[kMaxBodies];                // rank of (depth, chain) among the bodies
  alignas(16) float team_rows[kMaxBodies][kTeamRow];
};

// Task targets of an instance's costs (Sec. IV-A), in a block of their own that
// the kernels read when they run, so a change between calls is one small
// stream-ordered write and cached launch tables stay valid.
struct DevTargets {
  float z_des;
  float v_des[3];
  float q_des[4];         // base orientation target (w, x, y, z)
  int32_t or_target;      // 0: identity target (the orientation term uses q_base directly)
  int32_t terminal_z_abs; // 1: terminal target height z_terminal
  float z_terminal;
};

// One MPC instance's view for one planning iteration.
struct DevInst {
  const DevModel* model;
  const float* sigma;    // [I][K] position std per iteration and knot
  const float* x0;       // [nq + nv]
  const float* nominal;  // [E] nominal knots for this iteration
  float* samples;        // [N][E] perturbed knots of every sample
  float* costs;          // [N]
  uint32_t* masks;       // [N][H] debug contact masks, or null
  const float* f0z;      // [nc] original contact order
  const float* q0;       // [nu]
  int32_t N, H, K, nu, E, iter, n_iters, cost_kind, lanes, weight_mode;
  const uint32_t* tick_ptr;  // device-resident tick of the instance
  uint32_t tick_value;       // used instead when use_tick_value != 0
  int32_t use_tick_value;
  uint32_t seed_lo, seed_hi;
  float dt, delta, lambda;
  float w_h, w_or, w_q, w_cv, w_cf, w_eff, w_H, w_ee, w_tau;
  const DevTargets* targets;  // the instance's task targets
  int32_t generate;      // 1: sample knots from the counter-based stream; 0: read samples
  int32_t store_samples; // with generate: 1 writes the sampled knots to samples (the
                         // update reads them); 0 leaves them to the update to regenerate
  int32_t spline_mode;   // 0 cubic Hermite, 1 natural cubic, 2 quadratic (position knots, zero velocity targets)
  int32_t wave_prio;     // issue priority (0..3) of the rollout wavefronts among those sharing a SIMD
  // verification only (read when masks is set): per-step records of the
  // rollouts with trace_map[n] >= 0, see trace_record
  float* trace;              // [traced][H + 1][nq + 2 nv + 2], or null
  const int32_t* trace_map;  // [N] record slot of sample n, or -1
};

// Per-instance state of the weighting/update stage.
struct DevUpdate {
  const float* costs;    // [N]
  const float* samples;  // [N][E] (read when regen is null)
  const DevInst* regen;  // the iteration's sampling descriptor: the update draws the
                         // samples' knots again from the counter-based stream (null:
                         // reads samples)
  const float* nominal_in;  // [E]
  float* nominal_out;    // [E]
  float* weights;        // [N] or null
  float* best_knots;     // [E] or null
  float* info;           // mppi_step_info (S_best, best_iter, n_nonfinite, all_nonfinite) or null
  float* best_state;     // [E + 5] running best knots, S_best, best_iter, counters, best sample of this call
  uint32_t* tick;        // advanced by one after the last iteration of a call
  float* partial;        // [update_parts(N)][E] per-part weighted sums (scratch)
  uint32_t* done;        // parts finished in the current launch (0 between launches)
  int32_t N, E, iter, weight_mode, first_iter, last_iter, parts;
  int32_t threads;       // workgroup size of the instance's update launches (update_shape)
  float lambda;
};

// One tick prefix of a batch: the instance's state carried `steps` control steps
// along its best trajectory (the prediction descriptor reads the measured state
// and the trajectory from the instance's buffers), written to state_out.
struct PredItem {
  const DevInst* inst;
  float* state_out;
  int32_t steps;
};
// One warm-start shift of a batch (see the shift kernel): in -> out.
struct ShiftItem {
  const float* in;
  float* out;
  int32_t K, nu, F, nsub, n_steps, spline_mode;
  float delta;
};

// Per-call outputs of an instance's update launch (null fields: not wanted).
struct UpdateOut {
  float* knots_out;         // nominal output of the last iteration
  float* best_out;          // best knots
  void* info_out;           // mppi_step_info
  const float* nominal_in;  // replaces the descriptor's nominal input
};

// The update splits an instance's samples into `parts` consecutive slices, one
// workgroup each; the last workgroup to finish sums the slices in order.
// Workgroup size of the small per-call kernels (staging copies, warm-start
// shifts): one wavefront, which finds room wherever one rollout wavefront has
// ended on a device full of rollouts.
constexpr int kShiftThreads = 64;
constexpr int kUpdThreads = 256;
constexpr int kUpdMaxParts = 64;
constexpr int kUpdMinSlice = 64;  // samples per part at least
__host__ __device__ inline int update_parts(int N) {
  const int p = (N + kUpdMinSlice - 1) / kUpdMinSlice;
  return p < 1 ? 1 : (p > kUpdMaxParts ? kUpdMaxParts : p);
}
// Workgroup size and parts of an instance's update.  Up to 1024 samples (the
// sizes served together with other instances' rollouts) the workgroups are one
// wavefront of 64 threads over slices of 16 samples: a wavefront needs the
// registers of one SIMD where a rollout wavefront has ended, while a 256-thread
// workgroup needs four of them on one compute unit, which a device full of
// rollouts rarely has.  Larger instances take 256 threads over slices of 64.
// The shape depends on N only, so an instance's sums are the same in every path.
struct UpdShape {
  int threads, parts;
};
__host__ __device__ inline UpdShape update_shape(int N) {
  if (N <= 1024) {
    const int p = (N + 15) / 16;
    return UpdShape{64, p < 1 ? 1 : (p > kUpdMaxParts ? kUpdMaxParts : p)};
  }
  return UpdShape{kUpdThreads, update_parts(N)};
}


// ---------------------------------------------------------------------------
// LDS layouts of the rollout kernels (floats), shared by host and device.
// ---------------------------------------------------------------------------
// Body schedule, one rollout group of G lanes:
//   slot[b][36] per body, 16-byte aligned and read/written as float4:
//               forward kinematics R(9) p(3) v(6) beta(6) in [0,24);
//               reused by the backward sweep for Ia(21) pa(6) in [0,27),
//               then by the forward sweep for a'(6) in [0,6)
//   pad[16]    : unused (keeps the groups' bank stagger)
//   knots[E]   : this rollout's knots
//   red[G]     : reduction scratch
// A slot is 36 floats (4 LDS banks past a multiple of 32), so the slots that
// the lanes of one level touch at once start in different banks; rollout groups
// are staggered by 16 banks.
constexpr int kSlot = 36;
__host__ __device__ inline int group_floats(int G, int E) {
  const int raw = G * kSlot + 16 + ((E + 3) & ~3) + ((G + 3) & ~3);
  const int want = G < 32 ? 16 : 0;
  return raw + ((want - raw % 32) + 64) % 32;
}

// Model table, staged once per work item at the start of a block's LDS:
//   [0,24)            unused (keeps the layout's LDS bank alignment)
//   [24,88)           modified diagonal of the natural cubic spline's slope
//                     system (K entries; spline mode 1)
//   [88,88+nc*kCt)    contact rows (position, nominal normal force, index)
// and, for the chain schedule only, the body rows and the chain-body table.
constexpr int kTabSpline = 24;
constexpr int kTabContacts = 88;
__host__ __device__ inline int body_table_floats(int nc) { return kTabContacts + nc * kCt; }

// Body schedule: the model table is followed by every body's joint-rotation
// constants P0 | P1 | P2 (27 floats, rows 16-byte aligned), read once per
// physics step instead of being held in registers.
constexpr int kPRow = 28;
__host__ __device__ inline int body_sched_table_floats(int nb, int nc) { return body_table_floats(nc) + nb * kPRow; }

// Chain schedule: after the model table (with body rows and chain bodies), one
// region per rollout group:
//   rec[nb][kRec]   per-body record (see the chain kernel)
//   base[16]        world rotation (9) and position (3) of frame B
//   knots[E]        this rollout's knots
//   pub[nch][kPub]  articulated inertia and bias a chain's first body hands to
//                   its parent on another chain
//   att[natt][kAtt] frame (R p v beta) and a' of a body other chains hang off
//   red[GC]         reduction scratch
constexpr int kRec = 36;
constexpr int kPub = 28;
constexpr int kAtt = 32;
__host__ __device__ inline int chain_table_floats(int nb, int nc) {
  return body_table_floats(nc) + nb * kRow + kMaxChains * kMaxLevels;
}
__host__ __device__ inline int chain_group_floats(int GC, int nb, int E, int nch, int natt) {
  const int raw = nb * kRec + 16 + ((E + 3) & ~3) + nch * kPub + natt * kAtt + GC;
  const int r4 = (raw + 3) & ~3;
  return r4 + ((20 - r4 % 32) + 32) % 32;  // 16-byte aligned groups, staggered across LDS banks
}

// Team schedule: after the model table (then the team constants [slots][60] and
// the slot of chain c's body at depth d [kMaxChains][kMaxLevels] as integer
// bits), one region per rollout group (ns = slots = bodies):
//   br[ns][8]       per body: cos q, sin q, qd, tau | PD gain, qdd
//   fr[ns][28]      per body, lane k at 8k: rotated row of R, p, v (2), beta (2)
//   lr[ns][28]      lane k at 8k: e, axis, c (2) | U (2), 1/D, u
//   ir[ns][60]      lane k at 20k: articulated inertia rows (A, B, column of B, C;
//                   rotated) and bias (2)
//   pr[nch][60]     the same, carried to its parent by a chain's first body
//   ar[ns][8]       lane k at 2k: acceleration (2) of a body other chains hang off
//   bs[32]          frame B (R 9, p 3), base twist (6), base a' (6)
//   gr[60]          the base's articulated inertia rows, for its solve
//   knots[E], red[G]
__host__ __device__ inline int team_table_floats(int ns, int nc) {
  return body_table_floats(nc) + ns * kTeamSlot + kMaxChains * kMaxLevels;
}
struct TeamLayout {
  int br, fr, lr, ir, pr, ar, bs, gr, knots, red, total;
};
__host__ __device__ inline TeamLayout team_layout(int G, int ns, int E, int nch) {
  TeamLayout t;
  int o = 0;
  t.br = o; o += ns * 8;
  t.fr = o; o += ns * kFrSlot;
  t.lr = o; o += ns * kFrSlot;
  t.ir = o; o += ns * kTeamSlot;
  t.pr = o; o += nch * kTeamSlot;
  t.ar = o; o += ns * 8;
  t.bs = o; o += 32;
  t.gr = o; o += kTeamSlot;
  t.knots = o; o += (E + 3) & ~3;
  t.red = o; o += (G + 3) & ~3;
  t.total = o + ((16 - o % 32) + 32) % 32;  // 16-byte aligned groups, staggered across LDS banks
  return t;
}

}  // namespace mppi
