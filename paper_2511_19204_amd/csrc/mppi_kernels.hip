// mppi_kernels.hip -- gfx950 kernels of the MPPI hot path.
//
// Rollout kernel: G lanes per rollout (G in {4, 8, 16, 32, 64}), 64/G
// rollouts per wavefront, one lane per rigid body (= one actuated joint).
// Spatial quantities use the axes of the instantaneous base frame B (world
// axes for a fixed base) about each body's own joint origin, so a child's
// articulated inertia reaches its parent by a pure translation; the tree is
// swept level by level through LDS.  The kernel fuses, per rollout: counter-based sampling of
// the knots (Alg. 1 sampling step, eq. vel-clamp), then H control steps of
// Hermite reference (eq. hermite_segment), PD law (eq. pd-controller), soft
// contact, articulated-body forward dynamics, running cost (Sec. IV-A) and a
// linearly implicit Euler step, and finally the terminal cost.
//
// Update kernel: one workgroup per instance; min / max / argmin of the costs,
// min-max normalised softmax weights (eq. softmax_minmax; eq. omega-weights in
// raw mode), the weighted knot average (eq. update-nominal carried to the
// knots) and best-sample tracking (Sec. III-D).  Every reduction runs in a
// fixed order, so results do not depend on launch shape or co-scheduled work.

#include "mppi_dev.hpp"

namespace mppi {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

__device__ __forceinline__ float u01(uint32_t x) { return ((float)(x >> 9) + 0.5f) * 0x1p-23f; }

// 1-ulp hardware reciprocal and reciprocal square root (v_rcp_f32 / v_rsq_f32),
// used where a correctly rounded quotient is not required
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// packed symmetric 6x6, upper triangle row by row
__host__ __device__ constexpr int SI(int i, int j) {
  return i <= j ? i * 6 - i * (i - 1) / 2 + (j - i) : j * 6 - j * (j - 1) / 2 + (i - j);
}

__device__ __forceinline__ void sym6_mv(const float* A, const float* x, float* y) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 6; ++j) s = fmaf(A[SI(i, j)], x[j], s);
    y[i] = s;
  }
}

__device__ __forceinline__ void cross3(const float* a, const float* b, float* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// rotation matrix of a unit quaternion (w, x, y, z), row-major
__device__ __forceinline__ void quat_R(const float* q, float* R) {
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}

// LDS layout of one rollout group (floats):
//   slot[b][29] per body: forward kinematics R(9) p(3) v(6) beta(6);
//                         reused by the backward sweep for Ia(21) pa(6),
//                         then by the forward sweep for a'(6)
//   base[16]   : world rotation (9) and position (3) of frame B
//   knots[E]   : this rollout's knots
//   red[G]     : reduction scratch
// The slot stride is odd and a group's size is padded to G (mod 32) floats, so
// the 64 lanes of a wavefront (64/G groups) touch distinct LDS banks.
constexpr int kSlot = 29;
__host__ __device__ inline int group_floats(int G, int E) {
  const int raw = G * kSlot + 16 + ((E + 3) & ~3) + G;
  const int want = G < 32 ? G : 0;
  return raw + ((want - raw % 32) + 64) % 32;
}

// ---------------------------------------------------------------------------
// Per-lane physics of one step.  Lane b (< nb) owns body b and its joint.
//
// Frames: every body's spatial quantities are taken about its own joint origin
// p_b with the axes of the base frame B (world axes for a fixed base).  All
// these frames are inertial at the instant, so the articulated-body recursions
// keep their textbook form, while parent <-> child transforms reduce to pure
// translations by e_b = p_b - p_parent and lever arms stay one link long
// (referring everything to the base origin instead loses about three digits
// in float on a 6-deep leg).
// ---------------------------------------------------------------------------
struct StepIO {
  // inputs
  float q, v;          // joint state (revolute lanes)
  float bq[7], bv[6];  // base state (lane 0 of a floating-base group)
  float qref, vref;    // reference (revolute lanes)
  float dt;
  // outputs
  float qdd;           // joint acceleration
  float ba[6];         // base spatial acceleration, base coordinates (lane 0)
  float tau;           // clipped PD torque
  float cost;          // running-cost terms of this lane (when want_cost)
  uint32_t mask;       // contact activity bits of this lane's contacts
};

// Per-lane constants of the body (and joint) a lane owns, loaded once per kernel.
struct BodyConst {
  float P[27];        // joint rotation C(q) = P0 + cos q P1 + sin q P2
  float p_tree[3], axis_p[3], com[3], Ic[6];
  float mass, kp, kd, taumax, arm;
  int parent, depth, n_child, c_begin, c_count;
};

__device__ __forceinline__ void load_body(const DevModel& M, int b, bool body_lane, BodyConst& c) {
  const int bb = body_lane ? b : 0;
  const int j = bb - M.fb;
  const bool joint = body_lane && j >= 0;
#pragma unroll
  for (int k = 0; k < 27; ++k) c.P[k] = M.P[bb][k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c.p_tree[k] = M.p_tree[bb][k];
    c.axis_p[k] = M.axis_p[bb][k];
    c.com[k] = M.com[bb][k];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) c.Ic[k] = M.Ic[bb][k];
  c.mass = M.mass[bb];
  c.kp = joint ? M.kp[j] : 0.f;
  c.kd = joint ? M.kd[j] : 0.f;
  c.taumax = joint ? M.taumax[j] : 0.f;
  c.arm = joint ? M.arm[j] : 0.f;
  c.parent = M.parent[bb];
  c.depth = body_lane ? M.depth[bb] : -1;
  c.n_child = body_lane ? M.n_child[bb] : 0;
  c.c_begin = M.c_begin[bb];
  c.c_count = body_lane ? M.c_count[bb] : 0;
}

// motion vector m given about point O, re-expressed about O + e: (w, v + w x e)
__device__ __forceinline__ void shift_motion(const float* m, const float* e, float* out) {
  float we[3];
  cross3(m, e, we);
  out[0] = m[0]; out[1] = m[1]; out[2] = m[2];
  out[3] = m[3] + we[0]; out[4] = m[4] + we[1]; out[5] = m[5] + we[2];
}

// Articulated inertia I (packed) about the child origin carried to the parent
// origin, e = child origin - parent origin: with E = e^x,
// A' = A - B E - (B E)^T - E C E,  B' = B + E C,  C' = C.
__device__ __forceinline__ void shift_inertia_to_parent(const float* I, const float* e, float* O) {
  float B[9], C[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      B[r * 3 + c] = I[SI(r, c + 3)];
      C[r * 3 + c] = I[SI(r + 3, c + 3)];
    }
  // BE: row r of B crossed with e
  float BE[9];
#pragma unroll
  for (int r = 0; r < 3; ++r) cross3(B + r * 3, e, BE + r * 3);
  // EC: column k of C is e x C[:, k]
  float EC[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float col[3] = {C[k], C[3 + k], C[6 + k]};
    float o[3];
    cross3(e, col, o);
    EC[k] = o[0]; EC[3 + k] = o[1]; EC[6 + k] = o[2];
  }
  // ECE: row r of EC crossed with e
  float ECE[9];
#pragma unroll
  for (int r = 0; r < 3; ++r) cross3(EC + r * 3, e, ECE + r * 3);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = r; c < 3; ++c) O[SI(r, c)] = I[SI(r, c)] - BE[r * 3 + c] - BE[c * 3 + r] - ECE[r * 3 + c];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) O[SI(r, c + 3)] = B[r * 3 + c] + EC[r * 3 + c];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = r; c < 3; ++c) O[SI(r + 3, c + 3)] = I[SI(r + 3, c + 3)];
}

// terminal = true evaluates only the kinematics and the end-effector height term
// of the terminal cost (end-effector task) at the current state.
template <int G>
__device__ void physics_step(const DevModel& M, const BodyConst& bc, const DevInst* I, float* __restrict__ gs,
                             int b, bool body_lane, StepIO& io, bool want_cost, bool terminal = false) {
  float* slots = gs;
  float* base = gs + G * kSlot;
  const int fb = M.fb;
  const bool is_base = body_lane && fb && b == 0;
  const bool is_joint = body_lane && !is_base;
  const int j = b - fb;

  // ---- PD law (linearly implicit gain on unsaturated joints)
  float tau = 0.f, gain = 0.f;
  if (is_joint) {
    const float t = bc.kp * (io.qref - io.q) + bc.kd * (io.vref - io.v);
    const float tm = bc.taumax;
    if (t >= tm) {
      tau = tm;
    } else if (t <= -tm) {
      tau = -tm;
    } else {
      tau = t;
      gain = io.dt * (bc.kd + io.dt * bc.kp);
    }
  }
  io.tau = tau;

  // ---- frame B: world pose of the base; body 0 slot = identity frame with the base twist
  if (is_base) {
    float R[9];
    quat_R(io.bq + 3, R);
#pragma unroll
    for (int k = 0; k < 9; ++k) base[k] = R[k];
    base[9] = io.bq[0]; base[10] = io.bq[1]; base[11] = io.bq[2];
    float* s = slots;  // body 0
#pragma unroll
    for (int k = 0; k < 9; ++k) s[k] = (k % 4 == 0) ? 1.f : 0.f;
    s[9] = s[10] = s[11] = 0.f;
#pragma unroll
    for (int k = 0; k < 6; ++k) { s[12 + k] = io.bv[k]; s[18 + k] = 0.f; }
  }
  if (!fb && body_lane && b == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) base[k] = (k % 4 == 0) ? 1.f : 0.f;
    base[9] = base[10] = base[11] = 0.f;
  }
  wave_sync();

  // ---- forward kinematics, level by level (slot: R, p, v, beta about the body origin)
  float R[9], p[3], e[3], ax[3], v[6], c[6], beta[6];
  const int depth = bc.depth;
  if (is_base) {
#pragma unroll
    for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.f : 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) { p[k] = 0.f; e[k] = 0.f; ax[k] = 0.f; }
#pragma unroll
    for (int k = 0; k < 6; ++k) { v[k] = io.bv[k]; c[k] = 0.f; beta[k] = 0.f; }
  }
  float cq = 0.f, sq = 0.f;
  if (is_joint) sincosf(io.q, &sq, &cq);
  for (int d = 1; d <= M.max_depth; ++d) {
    if (is_joint && depth == d) {
      const int lam = bc.parent;
      float Rl[9], pl[3], vl[6], bl[6];
      if (lam >= 0) {
        const float* s = slots + lam * kSlot;
#pragma unroll
        for (int k = 0; k < 9; ++k) Rl[k] = s[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) pl[k] = s[9 + k];
#pragma unroll
        for (int k = 0; k < 6; ++k) { vl[k] = s[12 + k]; bl[k] = s[18 + k]; }
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) Rl[k] = (k % 4 == 0) ? 1.f : 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) pl[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) { vl[k] = 0.f; bl[k] = 0.f; }
      }
      const float* P = bc.P;
      float C[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) C[k] = P[k] + cq * P[9 + k] + sq * P[18 + k];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
          R[r * 3 + cc] = Rl[r * 3 + 0] * C[0 * 3 + cc] + Rl[r * 3 + 1] * C[1 * 3 + cc] + Rl[r * 3 + 2] * C[2 * 3 + cc];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        e[r] = Rl[r * 3 + 0] * bc.p_tree[0] + Rl[r * 3 + 1] * bc.p_tree[1] + Rl[r * 3 + 2] * bc.p_tree[2];
        p[r] = pl[r] + e[r];
        ax[r] = Rl[r * 3 + 0] * bc.axis_p[0] + Rl[r * 3 + 1] * bc.axis_p[1] + Rl[r * 3 + 2] * bc.axis_p[2];
      }
      // v = shift(v_parent) + S qd with S = (axis, 0) about the joint origin
      shift_motion(vl, e, v);
      v[0] += ax[0] * io.v; v[1] += ax[1] * io.v; v[2] += ax[2] * io.v;
      // c = v x_m (S qd) = (w x a qd, v_lin x a qd)
      const float aq[3] = {ax[0] * io.v, ax[1] * io.v, ax[2] * io.v};
      cross3(v, aq, c);
      cross3(v + 3, aq, c + 3);
      float bs[6];
      shift_motion(bl, e, bs);
#pragma unroll
      for (int k = 0; k < 6; ++k) beta[k] = bs[k] + c[k];
      float* s = slots + b * kSlot;
#pragma unroll
      for (int k = 0; k < 9; ++k) s[k] = R[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) s[9 + k] = p[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) { s[12 + k] = v[k]; s[18 + k] = beta[k]; }
    }
    wave_sync();
  }

  // ---- rigid-body inertia, bias force, contacts (all body lanes in parallel)
  float IA[21], pA[6];
  float lane_cost = 0.f;
  uint32_t mask = 0u;
  float Rb[9], pb[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rb[k] = base[k];
  pb[0] = base[9]; pb[1] = base[10]; pb[2] = base[11];
  if (terminal) {
    if (body_lane && I->cost_kind == 0 && b == M.ee_body) {
      float xe[3];
#pragma unroll
      for (int r = 0; r < 3; ++r)
        xe[r] = p[r] + R[r * 3 + 0] * M.ee_pos[0] + R[r * 3 + 1] * M.ee_pos[1] + R[r * 3 + 2] * M.ee_pos[2];
      const float dz = pb[2] + Rb[6] * xe[0] + Rb[7] * xe[1] + Rb[8] * xe[2] - I->z_des;
      lane_cost = I->w_ee * dz * dz;
    }
    io.cost = lane_cost;
    io.mask = 0u;
    wave_sync();
    return;
  }
  const float g = M.g;
  // gravity as a spatial acceleration in B axes: (0, Rb^T (0, 0, -g)), the same about any origin
  const float agl[3] = {-g * Rb[6], -g * Rb[7], -g * Rb[8]};
  if (body_lane) {
    if (is_base) {
#pragma unroll
      for (int k = 0; k < 21; ++k) IA[k] = M.base_I[k];
    } else {
      const float m = bc.mass;
      float cw[3];
      const float cb[3] = {bc.com[0], bc.com[1], bc.com[2]};
#pragma unroll
      for (int r = 0; r < 3; ++r) cw[r] = R[r * 3 + 0] * cb[0] + R[r * 3 + 1] * cb[1] + R[r * 3 + 2] * cb[2];
      const float* Ic = bc.Ic;
      const float Ib[9] = {Ic[0], Ic[3], Ic[4], Ic[3], Ic[1], Ic[5], Ic[4], Ic[5], Ic[2]};
      float RI[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
          RI[r * 3 + cc] = R[r * 3 + 0] * Ib[0 * 3 + cc] + R[r * 3 + 1] * Ib[1 * 3 + cc] + R[r * 3 + 2] * Ib[2 * 3 + cc];
      const float c2 = cw[0] * cw[0] + cw[1] * cw[1] + cw[2] * cw[2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int cc = r; cc < 3; ++cc) {
          const float iw = RI[r * 3 + 0] * R[cc * 3 + 0] + RI[r * 3 + 1] * R[cc * 3 + 1] + RI[r * 3 + 2] * R[cc * 3 + 2];
          IA[SI(r, cc)] = iw + m * ((r == cc ? c2 : 0.f) - cw[r] * cw[cc]);
        }
      IA[SI(0, 3)] = 0.f;        IA[SI(0, 4)] = -m * cw[2]; IA[SI(0, 5)] = m * cw[1];
      IA[SI(1, 3)] = m * cw[2];  IA[SI(1, 4)] = 0.f;        IA[SI(1, 5)] = -m * cw[0];
      IA[SI(2, 3)] = -m * cw[1]; IA[SI(2, 4)] = m * cw[0];  IA[SI(2, 5)] = 0.f;
      IA[SI(3, 3)] = m; IA[SI(3, 4)] = 0.f; IA[SI(3, 5)] = 0.f;
      IA[SI(4, 4)] = m; IA[SI(4, 5)] = 0.f; IA[SI(5, 5)] = m;
    }
    // bias force v x_f (I v)
    float h[6];
    sym6_mv(IA, v, h);
    float t0[3], t1[3], t2[3];
    cross3(v, h, t0);
    cross3(v + 3, h + 3, t1);
    cross3(v, h + 3, t2);
    pA[0] = t0[0] + t1[0]; pA[1] = t0[1] + t1[1]; pA[2] = t0[2] + t1[2];
    pA[3] = t2[0]; pA[4] = t2[1]; pA[5] = t2[2];

    // contacts carried by this body (point x relative to the body origin)
    const int c0 = bc.c_begin, cn = bc.c_count;
    for (int ci = c0; ci < c0 + cn; ++ci) {
      const float r0 = M.cpos[ci][0], r1 = M.cpos[ci][1], r2 = M.cpos[ci][2];
      float x[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) x[r] = R[r * 3 + 0] * r0 + R[r * 3 + 1] * r1 + R[r * 3 + 2] * r2;
      float wx[3];
      cross3(v, x, wx);
      const float vB[3] = {v[3] + wx[0], v[4] + wx[1], v[5] + wx[2]};
      const float xB[3] = {p[0] + x[0], p[1] + x[1], p[2] + x[2]};
      float pw[3], vw[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        pw[r] = pb[r] + Rb[r * 3 + 0] * xB[0] + Rb[r * 3 + 1] * xB[1] + Rb[r * 3 + 2] * xB[2];
        vw[r] = Rb[r * 3 + 0] * vB[0] + Rb[r * 3 + 1] * vB[1] + Rb[r * 3 + 2] * vB[2];
      }
      float fn = 0.f;
      if (pw[2] < 0.f) fn = fmaxf(0.f, -M.k * pw[2] - M.d * vw[2]);
      const float n2 = vw[0] * vw[0] + vw[1] * vw[1] + M.eps * M.eps;
      const float inv_nrm = rsq(n2);
      const float mfn = M.mu * fn * inv_nrm;
      const float fw[3] = {-mfn * vw[0], -mfn * vw[1], fn};
      float fB[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) fB[r] = Rb[0 * 3 + r] * fw[0] + Rb[1 * 3 + r] * fw[1] + Rb[2 * 3 + r] * fw[2];
      float xf[3];
      cross3(x, fB, xf);
      pA[0] -= xf[0]; pA[1] -= xf[1]; pA[2] -= xf[2];
      pA[3] -= fB[0]; pA[4] -= fB[1]; pA[5] -= fB[2];
      if (fn > 0.f) {
        mask |= 1u << M.corig[ci];
        // Velocity Jacobian of the contact law (world), tangential-normal coupling
        // dropped: D_w = a I + (d - a) z z^T - a w w^T with a = mu f_n / n and
        // w = v_t / n.  In B axes z -> zb (third row of Rb) and w -> ub = Rb^T w.
        const float aa = mfn;
        const float al = M.d - aa;
        const float zb[3] = {Rb[6], Rb[7], Rb[8]};
        const float wt[2] = {vw[0] * inv_nrm, vw[1] * inv_nrm};
        const float ub[3] = {Rb[0] * wt[0] + Rb[3] * wt[1], Rb[1] * wt[0] + Rb[4] * wt[1],
                             Rb[2] * wt[0] + Rb[5] * wt[1]};
        const float dt = io.dt;
        // added inertia dt P^T D P with P = [-x^x, 1]; with w1 = x x zb, w2 = x x ub:
        //   top-left  a (|x|^2 I - x x^T) + al w1 w1^T - a w2 w2^T
        //   top-right a x^x + al w1 zb^T - a w2 ub^T,   bottom-right D
        float w1[3], w2[3];
        cross3(x, zb, w1);
        cross3(x, ub, w2);
        const float x2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        const float dta = dt * aa, dtal = dt * al;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int cc = r; cc < 3; ++cc) {
            const float tl = aa * ((r == cc ? x2 : 0.f) - x[r] * x[cc]) + al * w1[r] * w1[cc] - aa * w2[r] * w2[cc];
            IA[SI(r, cc)] += dt * tl;
            const float br = (r == cc ? aa : 0.f) + al * zb[r] * zb[cc] - aa * ub[r] * ub[cc];
            IA[SI(r + 3, cc + 3)] += dt * br;
          }
        const float Xm[9] = {0.f, -x[2], x[1], x[2], 0.f, -x[0], -x[1], x[0], 0.f};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int cc = 0; cc < 3; ++cc)
            IA[SI(r, cc + 3)] += dta * Xm[r * 3 + cc] + dtal * w1[r] * zb[cc] - dta * w2[r] * ub[cc];
        // bias of the added inertia: dt P^T D P (a_g - beta) = dt (x x Dw', Dw'), w' = P (a_g - beta)
        const float sa[3] = {-beta[0], -beta[1], -beta[2]};
        const float sl[3] = {agl[0] - beta[3], agl[1] - beta[4], agl[2] - beta[5]};
        float sx[3];
        cross3(sa, x, sx);
        const float w3[3] = {sl[0] + sx[0], sl[1] + sx[1], sl[2] + sx[2]};
        const float zw = zb[0] * w3[0] + zb[1] * w3[1] + zb[2] * w3[2];
        const float uw = ub[0] * w3[0] + ub[1] * w3[1] + ub[2] * w3[2];
        float Dw3[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) Dw3[r] = aa * w3[r] + al * zw * zb[r] - aa * uw * ub[r];
        float xd[3];
        cross3(x, Dw3, xd);
        pA[0] += dt * xd[0]; pA[1] += dt * xd[1]; pA[2] += dt * xd[2];
        pA[3] += dt * Dw3[0]; pA[4] += dt * Dw3[1]; pA[5] += dt * Dw3[2];
      }
      if (want_cost && I->cost_kind == 1) {
        if (fn > 0.f) lane_cost += I->w_cv * (fabsf(vw[0]) + fabsf(vw[1]) + fabsf(vw[2]));
        lane_cost += I->w_cf * (fabsf(fw[0]) + fabsf(fw[1]) + fabsf(fw[2] - I->f0z[M.corig[ci]]));
      }
    }
    if (want_cost) {
      if (I->cost_kind == 1) {
        if (is_base) {
          const float* qt = io.bq + 3;
          const float vn = sqrtf(qt[1] * qt[1] + qt[2] * qt[2] + qt[3] * qt[3]);
          const float phi = 2.f * atan2f(vn, fabsf(qt[0]));
          lane_cost += I->w_h * fabsf(io.bq[2] - I->z_des) + I->w_or * phi * phi;
        }
        if (is_joint) {
          const float eq = io.q - I->q0[j];
          lane_cost += I->w_q * eq * eq + I->w_eff * tau * tau;
        }
      } else {
        if (is_joint) lane_cost += I->w_tau * tau * tau;
        if (b == M.ee_body) {
          float xe[3];
#pragma unroll
          for (int r = 0; r < 3; ++r)
            xe[r] = p[r] + R[r * 3 + 0] * M.ee_pos[0] + R[r * 3 + 1] * M.ee_pos[1] + R[r * 3 + 2] * M.ee_pos[2];
          const float dz = pb[2] + Rb[6] * xe[0] + Rb[7] * xe[1] + Rb[8] * xe[2] - I->z_des;
          lane_cost += I->w_ee * dz * dz;
        }
      }
    }
  }
  io.cost = lane_cost;
  io.mask = mask;
  wave_sync();

  // ---- backward sweep, leaves to root: each joint lane publishes its
  //      articulated inertia and bias already carried to its parent's origin
  float U[6], invD = 0.f, u = 0.f;
  for (int d = M.max_depth; d >= 0; --d) {
    if (body_lane && depth == d) {
      const int nch = bc.n_child;
      for (int k = 0; k < nch; ++k) {
        const float* s = slots + M.child[b][k] * kSlot;
#pragma unroll
        for (int q = 0; q < 21; ++q) IA[q] += s[q];
#pragma unroll
        for (int q = 0; q < 6; ++q) pA[q] += s[21 + q];
      }
      if (is_joint) {
        // S = (ax, 0): U = IA S, D = S.U + g, u = tau - S.pA
#pragma unroll
        for (int r = 0; r < 6; ++r)
          U[r] = IA[SI(r, 0)] * ax[0] + IA[SI(r, 1)] * ax[1] + IA[SI(r, 2)] * ax[2];
        const float Dv = (bc.arm + gain) + (ax[0] * U[0] + ax[1] * U[1] + ax[2] * U[2]);
        invD = rcp(Dv);
        u = tau - (ax[0] * pA[0] + ax[1] * pA[1] + ax[2] * pA[2]);
        float Ia[21];
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
          for (int cc = r; cc < 6; ++cc) Ia[SI(r, cc)] = IA[SI(r, cc)] - U[r] * U[cc] * invD;
        float Iac[6];
        sym6_mv(Ia, c, Iac);
        const float uD = u * invD;
        float pa[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) pa[q] = pA[q] + Iac[q] + U[q] * uD;
        float* s = slots + b * kSlot;
        float Ip[21];
        shift_inertia_to_parent(Ia, e, Ip);
#pragma unroll
        for (int q = 0; q < 21; ++q) s[q] = Ip[q];
        float ef[3];
        cross3(e, pa + 3, ef);
        s[21] = pa[0] + ef[0]; s[22] = pa[1] + ef[1]; s[23] = pa[2] + ef[2];
        s[24] = pa[3]; s[25] = pa[4]; s[26] = pa[5];
      }
    }
    wave_sync();
  }

  // ---- root: floating base solves IA0 a0' = -pA0 (Cholesky); fixed roots use -a_g
  if (is_base) {
    float L[21], invL[6];
#pragma unroll
    for (int q = 0; q < 21; ++q) L[q] = IA[q];
    // in-place Cholesky of the packed symmetric matrix (lower factor stored as L[SI(i,j)], j <= i)
#pragma unroll
    for (int jj = 0; jj < 6; ++jj) {
      float dsum = L[SI(jj, jj)];
#pragma unroll
      for (int k = 0; k < jj; ++k) dsum -= L[SI(jj, k)] * L[SI(jj, k)];
      const float inv = rsq(dsum);
      invL[jj] = inv;
      L[SI(jj, jj)] = dsum * inv;
#pragma unroll
      for (int i = jj + 1; i < 6; ++i) {
        float sm = L[SI(i, jj)];
#pragma unroll
        for (int k = 0; k < jj; ++k) sm -= L[SI(i, k)] * L[SI(jj, k)];
        L[SI(i, jj)] = sm * inv;
      }
    }
    float y[6], a0[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      float sm = -pA[i];
#pragma unroll
      for (int k = 0; k < i; ++k) sm -= L[SI(i, k)] * y[k];
      y[i] = sm * invL[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      float sm = y[i];
#pragma unroll
      for (int k = i + 1; k < 6; ++k) sm -= L[SI(k, i)] * a0[k];
      a0[i] = sm * invL[i];
    }
    float* s0 = slots;
#pragma unroll
    for (int q = 0; q < 6; ++q) s0[q] = a0[q];
    io.ba[0] = a0[0]; io.ba[1] = a0[1]; io.ba[2] = a0[2];
    io.ba[3] = a0[3] + agl[0]; io.ba[4] = a0[4] + agl[1]; io.ba[5] = a0[5] + agl[2];
  }
  wave_sync();

  // ---- forward sweep: accelerations, root to leaves
  float qdd = 0.f;
  for (int d = 1; d <= M.max_depth; ++d) {
    if (is_joint && depth == d) {
      const int lam = bc.parent;
      float al[6];
      if (lam >= 0) {
        const float* s = slots + lam * kSlot;
#pragma unroll
        for (int q = 0; q < 6; ++q) al[q] = s[q];
      } else {
        // fixed world: a' = -a_g = (0, 0, 0, 0, 0, g); its angular part is zero, so no shift term
        al[0] = al[1] = al[2] = 0.f; al[3] = 0.f; al[4] = 0.f; al[5] = g;
      }
      float a[6];
      shift_motion(al, e, a);
#pragma unroll
      for (int q = 0; q < 6; ++q) a[q] += c[q];
      float Ua = 0.f;
#pragma unroll
      for (int q = 0; q < 6; ++q) Ua = fmaf(U[q], a[q], Ua);
      qdd = (u - Ua) * invD;
      float* s = slots + b * kSlot;
      s[0] = a[0] + ax[0] * qdd; s[1] = a[1] + ax[1] * qdd; s[2] = a[2] + ax[2] * qdd;
      s[3] = a[3]; s[4] = a[4]; s[5] = a[5];
    }
    wave_sync();
  }
  io.qdd = qdd;
}

// ---------------------------------------------------------------------------
// Knot sampling for one rollout group: counter-based normals, perturbation,
// position clip and bound-aware velocity clamp.
// ---------------------------------------------------------------------------
template <int G>
__device__ void sample_group(const DevModel& M, const DevInst& I, int n, int l, float* knots, bool valid) {
  const int K = I.K, nu = I.nu, KU = K * nu;
  const int nblk = (KU + 1) / 2;
  const uint2 key = make_uint2(I.seed_lo, I.seed_hi);
  const float* sig = I.sigma + I.iter * K;
  const uint32_t tick = I.use_tick_value ? I.tick_value : *I.tick_ptr;
  for (int blk = l; blk < nblk; blk += G) {
    uint4 x = make_uint4(0u, 0u, 0u, 0u);
    if (n > 0) x = philox(make_uint4((uint32_t)blk, (uint32_t)n, (uint32_t)I.iter, tick), key);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int m = 2 * blk + half;
      if (m >= KU) break;
      const int k = m / nu, jj = m % nu;
      float zq = 0.f, zv = 0.f;
      if (n > 0) {
        const uint32_t xa = half ? x.z : x.x, xb = half ? x.w : x.y;
        const float ua = u01(xa), ub = u01(xb);
        const float r = sqrtf(-2.f * logf(ua));
        zq = r * cospif(2.f * ub);
        zv = r * sinpif(2.f * ub);
      }
      const float sq = sig[k];
      const float sv = sq / I.delta;
      const float lo = M.qmin[jj], hi = M.qmax[jj];
      float tq = fmaf(sq, zq, I.nominal[m]);
      tq = fminf(fmaxf(tq, lo), hi);
      const float lim = 2.f * fminf(hi - tq, tq - lo) / I.delta;
      float tv = fmaf(sv, zv, I.nominal[KU + m]);
      tv = fminf(fmaxf(tv, -lim), lim);
      knots[m] = tq;
      knots[KU + m] = tv;
      if (valid) {
        I.samples[(size_t)n * I.E + m] = tq;
        I.samples[(size_t)n * I.E + KU + m] = tv;
      }
    }
  }
}

// Hermite reference of joint jj at fine step f of F (eq. hermite_segment and
// its time derivative); segment and local time from integer arithmetic.
__device__ __forceinline__ void hermite(const float* knots, int K, int nu, int F, float delta, float inv_delta,
                                        int f, int jj, float* qr, float* vr) {
  const int m = f * (K - 1);
  int seg = m / F;
  seg = seg < K - 2 ? seg : K - 2;
  const float s = (float)(m - seg * F) / (float)F;
  const float s2 = s * s, s3 = s2 * s;
  const float h00 = 2.f * s3 - 3.f * s2 + 1.f, h10 = s3 - 2.f * s2 + s, h01 = -2.f * s3 + 3.f * s2, h11 = s3 - s2;
  const float d00 = 6.f * s2 - 6.f * s, d10 = 3.f * s2 - 4.f * s + 1.f, d01 = -6.f * s2 + 6.f * s, d11 = 3.f * s2 - 2.f * s;
  const int KU = K * nu;
  const float q0 = knots[seg * nu + jj], q1 = knots[(seg + 1) * nu + jj];
  const float v0 = knots[KU + seg * nu + jj], v1 = knots[KU + (seg + 1) * nu + jj];
  *qr = h00 * q0 + h10 * delta * v0 + h01 * q1 + h11 * delta * v1;
  *vr = (d00 * q0 + d10 * delta * v0 + d01 * q1 + d11 * delta * v1) * inv_delta;
}

template <int G>
__device__ __forceinline__ float group_sum(float x, float* red, int l) {
  red[l] = x;
  wave_sync();
  float s = 0.f;
  if (l == 0)
    for (int k = 0; k < G; ++k) s += red[k];
  wave_sync();
  return s;
}

template <int G>
__device__ __forceinline__ uint32_t group_or(uint32_t x, float* red, int l) {
  uint32_t* r = reinterpret_cast<uint32_t*>(red);
  r[l] = x;
  wave_sync();
  uint32_t s = 0u;
  if (l == 0)
    for (int k = 0; k < G; ++k) s |= r[k];
  wave_sync();
  return s;
}

// semi-implicit Euler on the base: v += dt a, p += dt R(quat) v_lin, quat <- quat (x) exp(dt w)
__device__ __forceinline__ void integrate_base(float* bq, float* bv, const float* ba, float dt) {
#pragma unroll
  for (int k = 0; k < 6; ++k) bv[k] = fmaf(dt, ba[k], bv[k]);
  float R[9];
  quat_R(bq + 3, R);
#pragma unroll
  for (int r = 0; r < 3; ++r) bq[r] += dt * (R[r * 3 + 0] * bv[3] + R[r * 3 + 1] * bv[4] + R[r * 3 + 2] * bv[5]);
  const float wn = sqrtf(bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2]);
  float e0 = 1.f, e1 = 0.f, e2 = 0.f, e3 = 0.f;
  if (wn > 0.f) {
    const float th = 0.5f * wn * dt;
    float sn, cs;
    sincosf(th, &sn, &cs);
    const float k = sn * rcp(wn);
    e0 = cs; e1 = k * bv[0]; e2 = k * bv[1]; e3 = k * bv[2];
  }
  const float a0 = bq[3], a1 = bq[4], a2 = bq[5], a3 = bq[6];
  const float r0 = a0 * e0 - a1 * e1 - a2 * e2 - a3 * e3;
  const float r1 = a0 * e1 + a1 * e0 + a2 * e3 - a3 * e2;
  const float r2 = a0 * e2 - a1 * e3 + a2 * e0 + a3 * e1;
  const float r3 = a0 * e3 + a1 * e2 - a2 * e1 + a3 * e0;
  const float inv = rsq(r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
  bq[3] = r0 * inv; bq[4] = r1 * inv; bq[5] = r2 * inv; bq[6] = r3 * inv;
}

// ---------------------------------------------------------------------------
// Fused rollout of one work item: 64/G rollouts of one instance, samples
// w.y .. w.y + 64/G - 1 (those >= N are computed but not stored).
// ---------------------------------------------------------------------------
template <int G>
__device__ void rollout_item(const DevInst& I, int first, int group_stride, float* smem) {
  const int lane = threadIdx.x;
  const int grp = lane / G, l = lane % G;
  const DevModel& M = *I.model;
  const int n = first + grp;
  const bool valid = n < I.N;
  float* gs = smem + grp * group_stride;
  float* knots = gs + G * kSlot + 16;
  float* red = knots + ((I.E + 3) & ~3);

  // knots of this sample
  if (I.generate) {
    sample_group<G>(M, I, valid ? n : 0, l, knots, valid);
  } else {
    const float* src = I.samples + (size_t)(valid ? n : 0) * I.E;
    for (int e = l; e < I.E; e += G) knots[e] = src[e];
  }
  wave_sync();

  const int fb = M.fb, nb = M.nb, nq = fb ? 7 + M.nu : M.nu;
  const bool body_lane = l < nb;
  const int b = l;
  const bool is_joint = body_lane && !(fb && b == 0);
  const int j = b - fb;
  StepIO io;
  io.q = io.v = 0.f;
  if (is_joint) {
    io.q = I.x0[(fb ? 7 : 0) + j];
    io.v = I.x0[nq + (fb ? 6 : 0) + j];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) io.bq[k] = fb ? I.x0[k] : 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) io.bv[k] = fb ? I.x0[nq + k] : 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) io.ba[k] = 0.f;
  io.qref = io.vref = 0.f;

  const int nsub = M.nsub, H = I.H, F = H * nsub;
  io.dt = I.dt / (float)nsub;
  const float inv_delta = 1.f / I.delta;
  BodyConst bc;
  load_body(M, b, body_lane, bc);
  float acc = 0.f;
  for (int f = 0; f < F; ++f) {
    const bool control = (f % nsub) == 0;
    if (is_joint) hermite(knots, I.K, I.nu, F, I.delta, inv_delta, f, j, &io.qref, &io.vref);
    physics_step<G>(M, bc, &I, gs, b, body_lane, io, control);
    if (control) {
      acc += io.cost;
      if (I.masks) {
        const uint32_t mk = group_or<G>(io.mask, red, l);
        if (l == 0 && valid) I.masks[(size_t)n * H + f / nsub] = mk;
      }
    }
    if (is_joint) {
      io.v = fmaf(io.dt, io.qdd, io.v);
      io.q = fmaf(io.dt, io.v, io.q);
    }
    if (fb && b == 0) integrate_base(io.bq, io.bv, io.ba, io.dt);
  }

  // terminal cost
  if (I.cost_kind == 1) {
    if (fb && b == 0) {
      const float T = (float)H * I.dt;
      float e = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) e += fabsf(io.bq[k] - (I.x0[k] + I.v_des[k] * T));
      acc += I.w_H * e;
    }
  } else {
    // end-effector height at x_H
    physics_step<G>(M, bc, &I, gs, b, body_lane, io, false, true);
    acc += io.cost;
  }
  float S = group_sum<G>(acc, red, l);
  if (l == 0 && valid) {
    if (!isfinite(S)) S = INFINITY;
    I.costs[n] = S;
  }
  wave_sync();
}

// Block = one wavefront; work[blockIdx] = (instance, first sample) or, when work
// is null, instance 0 and sample blockIdx * 64/G.
template <int G>
__global__ __launch_bounds__(64) void rollout_kernel(const DevInst* __restrict__ insts, const int2* __restrict__ work,
                                                     int group_stride) {
  extern __shared__ float smem[];
  constexpr int R = 64 / G;
  const int2 w = work ? work[blockIdx.x] : make_int2(0, (int)blockIdx.x * R);
  rollout_item<G>(insts[w.x], w.y, group_stride, smem);
}

// Persistent form: a grid sized to the resident wavefronts; each wavefront takes
// work items from a device counter until the table is exhausted (every wavefront
// reaches that exit).  Which wavefront runs an item does not change its result.
template <int G>
__global__ __launch_bounds__(64) void rollout_persistent_kernel(const DevInst* __restrict__ insts,
                                                                const int2* __restrict__ work, int n_items,
                                                                unsigned int* __restrict__ counter, int group_stride) {
  extern __shared__ float smem[];
  for (;;) {
    int item = 0;
    if (threadIdx.x == 0) item = (int)atomicAdd(counter, 1u);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= n_items) break;
    const int2 w = work[item];
    rollout_item<G>(insts[w.x], w.y, group_stride, smem);
  }
}

__global__ void reset_counters(unsigned int* __restrict__ c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
}

// ---------------------------------------------------------------------------
// Weighting, update and best tracking: one 256-thread workgroup per instance.
// out (per call): the final nominal, best knots and info of the last iteration.
// ---------------------------------------------------------------------------
struct UpdateOut {
  float* knots_out;   // nominal output of the last iteration
  float* best_out;    // best knots or null
  void* info_out;     // mppi_step_info or null
};

constexpr int kUpdThreads = 1024;
constexpr int kUpdWaves = kUpdThreads / 64;
constexpr int kUpdChunk = 4096;  // samples whose weights sit in LDS at a time

// Block-wide reductions in a fixed order (tree over threads), deterministic.
__device__ __forceinline__ float block_sum(float x, float* buf) {
  const int t = threadIdx.x;
  buf[t] = x;
  __syncthreads();
  for (int off = kUpdThreads / 2; off > 0; off >>= 1) {
    if (t < off) buf[t] += buf[t + off];
    __syncthreads();
  }
  const float r = buf[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kUpdThreads) void update_kernel(const DevUpdate* __restrict__ ups,
                                                             const UpdateOut* __restrict__ outs, UpdateOut single) {
  const DevUpdate& U = ups[blockIdx.x];
  const int t = threadIdx.x, N = U.N, E = U.E;
  __shared__ float s_v[kUpdThreads];
  __shared__ int s_i[kUpdThreads];
  __shared__ float s_x[kUpdThreads];
  __shared__ float s_w[kUpdChunk];
  __shared__ float s_part[kUpdWaves][64];

  // 1. finite minimum (lowest index), maximum and count
  float mn = INFINITY, mx = -INFINITY;
  int arg = 0x7fffffff, nf = 0;
  for (int n = t; n < N; n += kUpdThreads) {
    const float S = U.costs[n];
    if (isfinite(S)) {
      ++nf;
      if (S < mn) { mn = S; arg = n; }
      mx = fmaxf(mx, S);
    }
  }
  s_v[t] = mn; s_i[t] = arg; s_x[t] = mx;
  __syncthreads();
  for (int off = kUpdThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      const float om = s_v[t + off];
      const int oi = s_i[t + off];
      if (om < s_v[t] || (om == s_v[t] && oi < s_i[t])) { s_v[t] = om; s_i[t] = oi; }
      s_x[t] = fmaxf(s_x[t], s_x[t + off]);
    }
    __syncthreads();
  }
  const float smin = s_v[0], smax = s_x[0];
  const int nstar = s_i[0];
  __syncthreads();
  const int nfin = (int)block_sum((float)nf, s_x);

  // 2. unnormalised weights e_n = exp(-S_hat / lambda) and their sum
  const float range = smax - smin;
  const float inv_range = (U.weight_mode == 0 && range > 0.f) ? 1.f / range : 0.f;
  const float inv_lam = 1.f / U.lambda;
  auto weight = [&](float S) -> float {
    if (!isfinite(S)) return 0.f;
    const float sh = U.weight_mode == 0 ? (S - smin) * inv_range : (S - smin);
    return expf(-sh * inv_lam);
  };
  float zs = 0.f;
  for (int n = t; n < N; n += kUpdThreads) zs += weight(U.costs[n]);
  const float Z = block_sum(zs, s_x);
  const float invZ = nfin > 0 ? 1.f / Z : 0.f;
  if (U.weights)
    for (int n = t; n < N; n += kUpdThreads) U.weights[n] = weight(U.costs[n]) * invZ;

  // 3. weighted knot average: waves split the samples, lanes the knot elements
  const UpdateOut* o = outs ? outs + blockIdx.x : &single;
  float* dst = (U.last_iter && o && o->knots_out) ? o->knots_out : U.nominal_out;
  const int wv = t / 64, ln = t % 64;
  const int n_e = (E + 63) / 64;
  // accumulate each element's sum across chunks in registers of wave 0 after the reduction
  for (int eb = 0; eb < n_e; ++eb) {
    const int e = eb * 64 + ln;
    float total = 0.f;
    for (int c0 = 0; c0 < N; c0 += kUpdChunk) {
      const int cn = min(kUpdChunk, N - c0);
      __syncthreads();
      for (int n = t; n < cn; n += kUpdThreads) s_w[n] = weight(U.costs[c0 + n]) * invZ;
      __syncthreads();
      float acc = 0.f;
      if (e < E && nfin > 0) {
        const float* col = U.samples + (size_t)c0 * E + e;
        int n = wv;
        for (; n + 3 * kUpdWaves < cn; n += 4 * kUpdWaves) {
          const float a0 = col[(size_t)n * E];
          const float a1 = col[(size_t)(n + kUpdWaves) * E];
          const float a2 = col[(size_t)(n + 2 * kUpdWaves) * E];
          const float a3 = col[(size_t)(n + 3 * kUpdWaves) * E];
          acc = fmaf(s_w[n], a0, acc);
          acc = fmaf(s_w[n + kUpdWaves], a1, acc);
          acc = fmaf(s_w[n + 2 * kUpdWaves], a2, acc);
          acc = fmaf(s_w[n + 3 * kUpdWaves], a3, acc);
        }
        for (; n < cn; n += kUpdWaves) acc = fmaf(s_w[n], col[(size_t)n * E], acc);
      }
      s_part[wv][ln] = acc;
      __syncthreads();
      if (wv == 0) {
        float sum = 0.f;
#pragma unroll
        for (int k = 0; k < kUpdWaves; ++k) sum += s_part[k][ln];
        total += sum;
      }
    }
    if (wv == 0 && e < E) dst[e] = nfin > 0 ? total : U.nominal_in[e];
  }
  __syncthreads();

  // 4. best-sample tracking across the iterations of this call
  float* bs = U.best_state;  // [E] knots, then S_best, best_iter, n_nonfinite, all_nonfinite
  if (U.first_iter) {
    for (int e = t; e < E; e += kUpdThreads) bs[e] = U.nominal_in[e];
    if (t == 0) {
      bs[E] = INFINITY;
      reinterpret_cast<int*>(bs)[E + 1] = -1;
      reinterpret_cast<int*>(bs)[E + 2] = 0;
      reinterpret_cast<int*>(bs)[E + 3] = 0;
    }
  }
  __syncthreads();
  const bool improve = nfin > 0 && U.costs[nstar] < bs[E];
  __syncthreads();
  if (improve)
    for (int e = t; e < E; e += kUpdThreads) bs[e] = U.samples[(size_t)nstar * E + e];
  __syncthreads();
  if (t == 0) {
    if (improve) {
      bs[E] = U.costs[nstar];
      reinterpret_cast<int*>(bs)[E + 1] = U.iter;
    }
    reinterpret_cast<int*>(bs)[E + 2] += N - nfin;
    reinterpret_cast<int*>(bs)[E + 3] += nfin == 0 ? 1 : 0;
  }
  __syncthreads();
  if (U.last_iter && o) {
    if (o->best_out)
      for (int e = t; e < E; e += kUpdThreads) o->best_out[e] = bs[e];
    if (t == 0 && o->info_out) {
      float* inf = reinterpret_cast<float*>(o->info_out);
      inf[0] = bs[E];
      reinterpret_cast<int*>(inf)[1] = reinterpret_cast<int*>(bs)[E + 1];
      reinterpret_cast<int*>(inf)[2] = reinterpret_cast<int*>(bs)[E + 2];
      reinterpret_cast<int*>(inf)[3] = reinterpret_cast<int*>(bs)[E + 3];
    }
  }
  if (U.last_iter && t == 0 && U.tick) U.tick[0] += 1u;
}

// Copy per-call inputs (state, warm-start knots) into instance buffers.
struct StageItem {
  const float* src;
  float* dst;
  int32_t count;
};
__global__ void stage_kernel(const StageItem* __restrict__ items) {
  const StageItem it = items[blockIdx.x];
  for (int i = threadIdx.x; i < it.count; i += blockDim.x) it.dst[i] = it.src[i];
}

// ---------------------------------------------------------------------------
// Verification kernels (same device functions as the product path)
// ---------------------------------------------------------------------------
__global__ void philox_kernel(const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ key,
                              uint32_t* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 r = philox(make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]),
                         make_uint2(key[2 * i], key[2 * i + 1]));
  out[4 * i] = r.x; out[4 * i + 1] = r.y; out[4 * i + 2] = r.z; out[4 * i + 3] = r.w;
}

template <int G>
__global__ __launch_bounds__(64) void sample_kernel(const DevInst* __restrict__ inst, int group_stride) {
  extern __shared__ float smem[];
  constexpr int R = 64 / G;
  const int lane = threadIdx.x, grp = lane / G, l = lane % G;
  const DevInst& I = *inst;
  const int n = blockIdx.x * R + grp;
  float* knots = smem + grp * group_stride + G * kSlot + 16;
  sample_group<G>(*I.model, I, n < I.N ? n : 0, l, knots, n < I.N);
}

template <int G>
__global__ __launch_bounds__(64) void dynamics_kernel(const DevModel* __restrict__ model, int n_states,
                                                      const float* __restrict__ q, const float* __restrict__ v,
                                                      const float* __restrict__ qref, const float* __restrict__ vref,
                                                      float dt, float* __restrict__ qdd, int group_stride) {
  extern __shared__ float smem[];
  constexpr int R = 64 / G;
  const int lane = threadIdx.x, grp = lane / G, l = lane % G;
  const DevModel& M = *model;
  const int s_raw = blockIdx.x * R + grp;
  const bool valid = s_raw < n_states;
  const int s = valid ? s_raw : 0;
  const int fb = M.fb, nu = M.nu, nq = fb ? 7 + nu : nu, nv = fb ? 6 + nu : nu;
  float* gs = smem + grp * group_stride;
  const bool body_lane = l < M.nb;
  const bool is_joint = body_lane && !(fb && l == 0);
  const int j = l - fb;
  StepIO io;
  io.q = is_joint ? q[(size_t)s * nq + (fb ? 7 : 0) + j] : 0.f;
  io.v = is_joint ? v[(size_t)s * nv + (fb ? 6 : 0) + j] : 0.f;
  io.qref = is_joint ? qref[(size_t)s * nu + j] : 0.f;
  io.vref = is_joint ? vref[(size_t)s * nu + j] : 0.f;
#pragma unroll
  for (int k = 0; k < 7; ++k) io.bq[k] = fb ? q[(size_t)s * nq + k] : 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) { io.bv[k] = fb ? v[(size_t)s * nv + k] : 0.f; io.ba[k] = 0.f; }
  io.dt = dt;
  BodyConst bc;
  load_body(M, l, body_lane, bc);
  physics_step<G>(M, bc, nullptr, gs, l, body_lane, io, false);
  if (!valid) return;
  if (is_joint) qdd[(size_t)s * nv + (fb ? 6 : 0) + j] = io.qdd;
  if (fb && l == 0)
    for (int k = 0; k < 6; ++k) qdd[(size_t)s * nv + k] = io.ba[k];
}

// explicit instantiations
#define MPPI_INST(G)                                                                                   \
  template __global__ void rollout_kernel<G>(const DevInst*, const int2*, int);                        \
  template __global__ void rollout_persistent_kernel<G>(const DevInst*, const int2*, int, unsigned int*, int); \
  template __global__ void sample_kernel<G>(const DevInst*, int);                                      \
  template __global__ void dynamics_kernel<G>(const DevModel*, int, const float*, const float*,        \
                                              const float*, const float*, float, float*, int);
MPPI_INST(4)
MPPI_INST(8)
MPPI_INST(16)
MPPI_INST(32)
MPPI_INST(64)
#undef MPPI_INST

}  // namespace mppi
