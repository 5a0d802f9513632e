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

// Kinematic tree in the layout the rollout lanes read: one entry per body,
// contacts sorted by body.  Precomputed on the host from mppi_model_desc:
//  * the joint rotation C(q) = R_tree Rot(axis, q) is stored as
//    C = P0 + cos(q) P1 + sin(q) P2 (Rodrigues' formula distributed over R_tree);
//  * axis_p = R_tree axis, the joint axis in the parent frame;
//  * base_I = spatial inertia of the base about its own origin (packed 6x6).
struct DevModel {
  int32_t nb, fb, nu, nc, nsub, ee_body, n_levels, max_depth;
  float k, d, mu, eps, g, mtot;
  float ee_pos[3];
  float base_I[21];
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
  float w_h, w_or, w_q, w_cv, w_cf, w_eff, w_H, w_ee, w_tau, z_des;
  float v_des[3];
  int32_t generate;      // 1: sample knots from the counter-based stream; 0: read samples
};

// Per-instance state of the weighting/update stage.
struct DevUpdate {
  const float* costs;    // [N]
  const float* samples;  // [N][E]
  const float* nominal_in;  // [E]
  float* nominal_out;    // [E]
  float* weights;        // [N] or null
  float* best_knots;     // [E] or null
  float* info;           // mppi_step_info (S_best, best_iter, n_nonfinite, all_nonfinite) or null
  float* best_state;     // [E + 4] running best knots, S_best, best_iter, counters of this call
  uint32_t* tick;        // advanced by one after the last iteration of a call
  int32_t N, E, iter, weight_mode, first_iter, last_iter;
  float lambda;
};

}  // namespace mppi
