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

// Branch-weight hint for a rare path when H holds (a compile-time constant),
// else the condition as is.  With one wavefront per SIMD every taken branch
// costs that wavefront an instruction refetch, so the legged and depth-6
// kernels ask for their rare paths to be laid out of line; the other kernels
// keep the default layout (with the hints their register allocation spills).  A macro: the hint
// has to sit in the branch's own condition.
#define MPPI_RARE(H, c) ((H) ? __builtin_expect(!!(c), 0) : !!(c))

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    // the 64-bit products give high and low words in one multiply each
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
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

// 16-byte LDS transfers of slot records (addresses are 16-byte aligned)
__device__ __forceinline__ void put4(float* d, float a, float b, float c, float e) {
  *reinterpret_cast<float4*>(d) = make_float4(a, b, c, e);
}
__device__ __forceinline__ float4 get4(const float* s) { return *reinterpret_cast<const float4*>(s); }

// frame record: R (9), p (3), v (6), beta (6)
__device__ __forceinline__ void put_frame(float* d, const float* R, const float* p, const float* v, const float* bt) {
  put4(d, R[0], R[1], R[2], R[3]);
  put4(d + 4, R[4], R[5], R[6], R[7]);
  put4(d + 8, R[8], p[0], p[1], p[2]);
  put4(d + 12, v[0], v[1], v[2], v[3]);
  put4(d + 16, v[4], v[5], bt[0], bt[1]);
  put4(d + 20, bt[2], bt[3], bt[4], bt[5]);
}
__device__ __forceinline__ void get_frame(const float* s, float* R, float* p, float* v, float* bt) {
  const float4 a = get4(s), b = get4(s + 4), c = get4(s + 8), d = get4(s + 12), e = get4(s + 16), f = get4(s + 20);
  R[0] = a.x; R[1] = a.y; R[2] = a.z; R[3] = a.w; R[4] = b.x; R[5] = b.y; R[6] = b.z; R[7] = b.w; R[8] = c.x;
  p[0] = c.y; p[1] = c.z; p[2] = c.w;
  v[0] = d.x; v[1] = d.y; v[2] = d.z; v[3] = d.w; v[4] = e.x; v[5] = e.y;
  bt[0] = e.z; bt[1] = e.w; bt[2] = f.x; bt[3] = f.y; bt[4] = f.z; bt[5] = f.w;
}
// articulated inertia (21, packed) and bias (6) record, one float of padding
__device__ __forceinline__ void put_art(float* d, const float* Ip, const float* pp) {
#pragma unroll
  for (int k = 0; k < 5; ++k) put4(d + 4 * k, Ip[4 * k], Ip[4 * k + 1], Ip[4 * k + 2], Ip[4 * k + 3]);
  put4(d + 20, Ip[20], pp[0], pp[1], pp[2]);
  put4(d + 24, pp[3], pp[4], pp[5], 0.f);
}
__device__ __forceinline__ void add_art(const float* s, float* IA, float* pA) {
  float t[28];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const float4 x = get4(s + 4 * k);
    t[4 * k] = x.x; t[4 * k + 1] = x.y; t[4 * k + 2] = x.z; t[4 * k + 3] = x.w;
  }
#pragma unroll
  for (int q = 0; q < 21; ++q) IA[q] += t[q];
#pragma unroll
  for (int q = 0; q < 6; ++q) pA[q] += t[21 + q];
}
// spatial acceleration record (6)
__device__ __forceinline__ void put_acc(float* d, const float* a) {
  put4(d, a[0], a[1], a[2], a[3]);
  *reinterpret_cast<float2*>(d + 4) = make_float2(a[4], a[5]);
}
__device__ __forceinline__ void get_acc(const float* s, float* a) {
  const float4 x = get4(s);
  const float2 y = *reinterpret_cast<const float2*>(s + 4);
  a[0] = x.x; a[1] = x.y; a[2] = x.z; a[3] = x.w; a[4] = y.x; a[5] = y.y;
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
  float bq[7], bv[6];  // base state (every lane of a floating-base rollout in the body schedule)
  float qref, vref;    // reference (revolute lanes)
  float dt;
  // outputs
  float qdd;           // joint acceleration
  float ba[6];         // base spatial acceleration, base coordinates (every lane of the rollout)
  float Rb[9];         // rotation of the base quaternion at the start of the step
  float tau;           // clipped PD torque
  float cost;          // running-cost terms of this lane (when want_cost)
  uint32_t mask;       // contact activity bits of this lane's contacts
};

// Per-lane constants of the body (and joint) a lane owns, loaded once per work item.
struct BodyConst {
  const float* P;     // joint rotation C(q) = P0 + cos q P1 + sin q P2, a row of the LDS table
  float p_tree[3], axis_p[3], com[3], Ic[6];
  float mass, kp, kd, taumax, arm, q0;
  int parent, depth, n_child, c_begin, c_count;
  float ct0[5];                 // first contact row: position (body frame), nominal normal force, index bits
  uint32_t child_lo, child_hi;  // children reached through LDS, 8 bits each, child-list order
  uint32_t flags;               // kAdjParent | kAdjChild | kFrameOut | kArtOut
};

// Transfers between a body and its first child in a depth-first numbering go
// through registers: the child (body b + 1) sits in the next lane, so one
// wavefront-wide shift by one lane moves a frame, an acceleration or an
// articulated inertia.  Other parent/child pairs go through the LDS slots.
constexpr uint32_t kAdjParent = 1u;  // joint body whose parent is the previous lane (a joint body)
constexpr uint32_t kAdjChild = 2u;   // first child is the next lane
constexpr uint32_t kFrameOut = 4u;   // joint body with a child that reads its frame and acceleration from LDS
constexpr uint32_t kArtOut = 8u;     // joint body whose parent reads its articulated inertia from LDS

__device__ __forceinline__ void load_body(const DevModel& M, const DevInst* I, int b, bool body_lane, const float* tab,
                                          BodyConst& c) {
  const int bb = body_lane ? b : 0;
  const int j = bb - M.fb;
  const bool joint = body_lane && j >= 0;
  c.P = tab + body_table_floats(M.nc) + bb * kPRow;
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
  c.q0 = (joint && I && I->cost_kind == 1) ? I->q0[j] : 0.f;
  c.parent = M.parent[bb];
  c.depth = body_lane ? M.depth[bb] : -1;
  c.c_begin = M.c_begin[bb];
  c.c_count = body_lane ? M.c_count[bb] : 0;
  {
    const float* ct = tab + kTabContacts + (c.c_count > 0 ? c.c_begin : 0) * kCt;
#pragma unroll
    for (int k = 0; k < 5; ++k) c.ct0[k] = ct[k];
  }
  // children are numbered after their parent in increasing order, so body b + 1,
  // when it is a child of b, is b's first child
  const int par = body_lane ? M.parent[bb] : -1;
  const int nch = body_lane ? M.n_child[bb] : 0;
  const bool adj_child = nch > 0 && M.child[bb][0] == bb + 1;
  c.flags = 0u;
  if (adj_child) c.flags |= kAdjChild;
  if (joint && par >= 0 && par == bb - 1 && !(M.fb && par == 0)) c.flags |= kAdjParent;
  if (joint && par >= 0 && bb != par + 1) c.flags |= kArtOut;
  c.n_child = 0;
  c.child_lo = c.child_hi = 0u;
  for (int k = 0; k < nch; ++k) {
    const int chb = M.child[bb][k];
    if (joint && chb != bb + 1) c.flags |= kFrameOut;
    if (k == 0 && adj_child) continue;
    const uint32_t ch = (uint32_t)chb & 0xffu;
    if (c.n_child < 4) c.child_lo |= ch << (8 * c.n_child);
    else c.child_hi |= ch << (8 * (c.n_child - 4));
    ++c.n_child;
  }
}
__device__ __forceinline__ int child_of(const BodyConst& c, int k) {
  return (int)(((k < 4 ? c.child_lo : c.child_hi) >> (8 * (k & 3))) & 0xffu);
}

// value held by the previous / next lane of the wavefront (DPP wave shift by one
// lane; every lane must be active; lanes past the wavefront's ends read 0)
__device__ __forceinline__ float from_prev_lane(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next_lane(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x130, 0xf, 0xf, true));
}
// value held by lane l + N of this lane's row of 16 lanes (DPP row shift;
// every lane must be active; lanes past the row's end read 0)
template <int N>
__device__ __forceinline__ float from_row_lane(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x100 + N, 0xf, 0xf, true));
}
// value held by the first lane of this lane's rollout group of G lanes (groups
// are aligned): for G = 16 a DPP broadcast of each row's lane 0
// (row_newbcast:0), for G = 4 a quad permutation (0, 0, 0, 0), else a swizzle
// in bit-mask mode that clears the low lane-index bits within each 32-lane
// half, or the first lane for a whole wavefront; every lane must be active
template <int G>
__device__ __forceinline__ float from_group_lane0(float x) {
  if constexpr (G == 64) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
  } else if constexpr (G == 16) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x150, 0xf, 0xf, false));
  } else if constexpr (G == 4) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x00, 0xf, 0xf, false));
  } else {
    constexpr int and_mask = 0x1f & ~(G - 1);
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x), and_mask));
  }
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
// C' = C,  B' = B + E C,  A' = A - B E - (B E)^T - E C E = A - B' E - (B E)^T
// (row r of X E is row r of X crossed with e).
__device__ __forceinline__ void shift_inertia_to_parent(const float* I, const float* e, float* O) {
  float B[9], C[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      B[r * 3 + c] = I[SI(r, c + 3)];
      C[r * 3 + c] = I[SI(r + 3, c + 3)];
    }
  // B' = B + E C: column k of E C is e x C[:, k]
  float Bp[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float col[3] = {C[k], C[3 + k], C[6 + k]};
    float o[3];
    cross3(e, col, o);
    Bp[k] = B[k] + o[0]; Bp[3 + k] = B[3 + k] + o[1]; Bp[6 + k] = B[6 + k] + o[2];
  }
  // (x cross e)[c] = x[c+1] e[c+2] - x[c+2] e[c+1]
  auto xe = [&](const float* x, int c) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    return x[c1] * e[c2] - x[c2] * e[c1];
  };
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = r; c < 3; ++c) O[SI(r, c)] = I[SI(r, c)] - xe(Bp + r * 3, c) - xe(B + c * 3, r);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) O[SI(r, c + 3)] = Bp[r * 3 + c];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = r; c < 3; ++c) O[SI(r + 3, c + 3)] = I[SI(r + 3, c + 3)];
}

// ---------------------------------------------------------------------------
// Per-body physics shared by both rollout schedules.  Each helper is the
// arithmetic of one body (or joint) in one phase; the schedules differ only in
// which lane runs it and where its operands come from, so they produce the
// same bits.
// ---------------------------------------------------------------------------

// PD law (eq. pd-controller) with the torque clip; on unsaturated joints the
// damping and stiffness act implicitly through the gain dt (Kd + dt Kp).
__device__ __forceinline__ void pd_law(float kp, float kd, float tm, float dt, float q, float v, float qref, float vref,
                                       float& tau, float& gain) {
  const float t = kp * (qref - q) + kd * (vref - v);
  const bool inside = t < tm && t > -tm;
  tau = fminf(fmaxf(t, -tm), tm);
  gain = inside ? dt * (kd + dt * kp) : 0.f;
}

// velocity-product acceleration c = v x_m (S qd) of a revolute joint, S = (ax, 0)
__device__ __forceinline__ void vel_product(const float* v, const float* ax, float qd, float* c) {
  const float aq[3] = {ax[0] * qd, ax[1] * qd, ax[2] * qd};
  cross3(v, aq, c);
  cross3(v + 3, aq, c + 3);
}

// Joint rotation C(q) = P0 + cos q P1 + sin q P2 (row-major 3x3) from the 27
// constants P0 | P1 | P2 (read as 28 floats from a 16-byte aligned address).
__device__ __forceinline__ void load_rotation_constants(const float* P, float* t) {
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const float4 x = *reinterpret_cast<const float4*>(P + 4 * k);
    t[4 * k] = x.x; t[4 * k + 1] = x.y; t[4 * k + 2] = x.z; t[4 * k + 3] = x.w;
  }
}
__device__ __forceinline__ void joint_rotation_of(const float* t, float cq, float sq, float* C) {
#pragma unroll
  for (int k = 0; k < 9; ++k) C[k] = t[k] + cq * t[9 + k] + sq * t[18 + k];
}
__device__ __forceinline__ void joint_rotation(const float* P, float cq, float sq, float* C) {
  float t[28];
  load_rotation_constants(P, t);
  joint_rotation_of(t, cq, sq, C);
}

// Forward kinematics of a revolute body from its parent's frame (Rl, pl), twist
// vl and bias acceleration bl, with joint rotation C: rotation R = Rl C, origin
// p, lever arm e = p - pl, axis ax (base axes), twist v, velocity product c and
// bias acceleration beta, all about the body's own origin.
__device__ __forceinline__ void fk_joint(const float* Rl, const float* pl, const float* vl, const float* bl,
                                         const float* C, const float* p_tree, const float* axis_p, float qd, float* R,
                                         float* p, float* e, float* ax, float* v, float* c, float* beta) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      R[r * 3 + cc] = Rl[r * 3 + 0] * C[0 * 3 + cc] + Rl[r * 3 + 1] * C[1 * 3 + cc] + Rl[r * 3 + 2] * C[2 * 3 + cc];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    e[r] = Rl[r * 3 + 0] * p_tree[0] + Rl[r * 3 + 1] * p_tree[1] + Rl[r * 3 + 2] * p_tree[2];
    p[r] = pl[r] + e[r];
    ax[r] = Rl[r * 3 + 0] * axis_p[0] + Rl[r * 3 + 1] * axis_p[1] + Rl[r * 3 + 2] * axis_p[2];
  }
  // v = shift(v_parent) + S qd with S = (axis, 0) about the joint origin
  shift_motion(vl, e, v);
  v[0] += ax[0] * qd; v[1] += ax[1] * qd; v[2] += ax[2] * qd;
  vel_product(v, ax, qd, c);
  float bs[6];
  shift_motion(bl, e, bs);
#pragma unroll
  for (int k = 0; k < 6; ++k) beta[k] = bs[k] + c[k];
}

// fk_joint for a child of the floating base, whose frame in base axes is the
// identity at the origin with twist bv and no bias acceleration: R = C(q),
// e = p = p_tree, ax = axis_p (the same values fk_joint gives for that parent).
__device__ __forceinline__ void fk_base_child(const float* bv, const float* C, const float* p_tree,
                                              const float* axis_p, float qd, float* R, float* p, float* e, float* ax,
                                              float* v, float* c, float* beta) {
#pragma unroll
  for (int k = 0; k < 9; ++k) R[k] = C[k];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    e[r] = p_tree[r];
    p[r] = p_tree[r];
    ax[r] = axis_p[r];
  }
  shift_motion(bv, e, v);
  v[0] += ax[0] * qd; v[1] += ax[1] * qd; v[2] += ax[2] * qd;
  vel_product(v, ax, qd, c);
#pragma unroll
  for (int k = 0; k < 6; ++k) beta[k] = c[k];
}

// Spatial inertia (packed) of a rigid body about its origin in base axes, from
// its rotation R, com and inertia Ic about the com (body frame) and mass m.
__device__ __forceinline__ void body_inertia(const float* R, const float* com, const float* Ic, float m, float* IA) {
  float cw[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) cw[r] = R[r * 3 + 0] * com[0] + R[r * 3 + 1] * com[1] + R[r * 3 + 2] * com[2];
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
__device__ __forceinline__ void bias_force(const float* IA, const float* v, float* pA) {
  float h[6];
  sym6_mv(IA, v, h);
  float t0[3], t1[3], t2[3];
  cross3(v, h, t0);
  cross3(v + 3, h + 3, t1);
  cross3(v, h + 3, t2);
  pA[0] = t0[0] + t1[0]; pA[1] = t0[1] + t1[1]; pA[2] = t0[2] + t1[2];
  pA[3] = t2[0]; pA[4] = t2[1]; pA[5] = t2[2];
}

// One soft contact point at r (body frame) on a body with frame (R, p), twist v
// and bias acceleration beta; frame B is (Rb, pb) in the world, agl is gravity
// in B axes.  Adds the contact force to the bias pA and, while the point
// penetrates, the linearly implicit damping/friction terms to IA and pA.
// Returns the normal force; vw and fw are the point's world velocity and force.
// Position-only spline variants (spline ablation, Sec. V): knot slopes dq/dt
// derived from the position knots and kept in the velocity block, so the curve
// is evaluated in Hermite form.  Natural cubic spline (mode 1): C2 at interior
// knots, zero end second derivatives, i.e. the tridiagonal system
// m_{k-1} + 4 m_k + m_{k+1} = 3 (q_{k+1} - q_{k-1}) / Delta with end rows
// (2, 1) and (1, 2); its eliminated diagonal depends on K only.  Quadratic
// spline (mode 2): m_0 = 0, m_{k+1} = 2 (q_{k+1} - q_k) / Delta - m_k.
__device__ __forceinline__ void natural_cubic_diagonal(int K, float* dg) {
  float d = 2.f;
  dg[0] = d;
  for (int k = 1; k < K; ++k) {
    const float w = 1.f / d;
    d = (k == K - 1 ? 2.f : 4.f) - w;
    dg[k] = d;
  }
}

// Slopes of joint jj for a knot vector in LDS (positions in [0, K nu),
// slopes written to [K nu, 2 K nu)); dg = natural_cubic_diagonal(K) for mode 1.
__device__ __forceinline__ void position_spline_slopes(int mode, int K, int nu, int jj, float delta, const float* dg,
                                                       float* knots) {
  const float* Q = knots;
  float* V = knots + K * nu;
  if (mode == 2) {
    float m = 0.f;
    V[jj] = m;
    for (int k = 0; k + 1 < K; ++k) {
      m = 2.f * (Q[(k + 1) * nu + jj] - Q[k * nu + jj]) / delta - m;
      V[(k + 1) * nu + jj] = m;
    }
    return;
  }
  // forward elimination (right-hand sides into V), then back substitution
  float prev = 0.f;
  for (int k = 0; k < K; ++k) {
    const float qa = Q[(k == 0 ? 0 : k - 1) * nu + jj], qb = Q[(k == K - 1 ? K - 1 : k + 1) * nu + jj];
    float r = 3.f * (qb - qa) / delta;
    if (k > 0) r -= (1.f / dg[k - 1]) * prev;
    V[k * nu + jj] = r;
    prev = r;
  }
  float next = V[(K - 1) * nu + jj] / dg[K - 1];
  V[(K - 1) * nu + jj] = next;
  for (int k = K - 2; k >= 0; --k) {
    next = (V[k * nu + jj] - next) / dg[k];
    V[k * nu + jj] = next;
  }
}

struct ContactLaw {
  float k, d, mu, eps;
};

// Model and instance scalars every step reads, loaded into registers once per
// work item (read through the model pointer inside the step loop, the compiler
// would reload them after every LDS store).
struct StepConst {
  int fb, max_depth, ee_body, cost_kind, K, nu, F, nsub, spline_mode;
  float g, dt, delta, inv_delta, inv_F;
  ContactLaw law;
  float ee_pos[3];
  float w_h, w_or, w_q, w_cv, w_cf, w_eff, w_ee, w_tau, z_des;
  int or_target;
  float q_des[4];
};
__device__ __forceinline__ StepConst load_step_const(const DevModel& M, const DevInst* I, float dt_override) {
  StepConst c;
  c.fb = M.fb; c.max_depth = M.max_depth; c.ee_body = M.ee_body; c.nsub = M.nsub;
  c.g = M.g;
  c.law = ContactLaw{M.k, M.d, M.mu, M.eps};
  c.ee_pos[0] = M.ee_pos[0]; c.ee_pos[1] = M.ee_pos[1]; c.ee_pos[2] = M.ee_pos[2];
  if (I) {
    c.cost_kind = I->cost_kind; c.K = I->K; c.nu = I->nu; c.F = I->H * M.nsub; c.spline_mode = I->spline_mode;
    c.dt = I->dt / (float)M.nsub;
    c.delta = I->delta; c.inv_delta = 1.f / I->delta; c.inv_F = 1.f / (float)c.F;
    c.w_h = I->w_h; c.w_or = I->w_or; c.w_q = I->w_q; c.w_cv = I->w_cv; c.w_cf = I->w_cf; c.w_eff = I->w_eff;
    const DevTargets& tg = *I->targets;
    c.w_ee = I->w_ee; c.w_tau = I->w_tau; c.z_des = tg.z_des;
    c.or_target = tg.or_target;
    c.q_des[0] = tg.q_des[0]; c.q_des[1] = tg.q_des[1]; c.q_des[2] = tg.q_des[2]; c.q_des[3] = tg.q_des[3];
  } else {
    c.cost_kind = -1; c.K = 2; c.nu = M.nu; c.F = 1; c.spline_mode = 0;
    c.dt = dt_override;
    c.delta = 1.f; c.inv_delta = 1.f; c.inv_F = 1.f;
    c.w_h = c.w_or = c.w_q = c.w_cv = c.w_cf = c.w_eff = c.w_ee = c.w_tau = c.z_des = 0.f;
    c.or_target = 0;
    c.q_des[0] = 1.f; c.q_des[1] = c.q_des[2] = c.q_des[3] = 0.f;
  }
  return c;
}

// Stage the model table (contact rows with the instance's nominal
// normal forces) into LDS with all 64 lanes of the wavefront.
__device__ __forceinline__ void stage_model_table(const DevModel& M, const DevInst* I, float* tab, int lane,
                                                  bool joint_rows = false) {
  const float* cs = &M.ctab[0][0];
  for (int i = lane; i < M.nc * kCt; i += 64) tab[kTabContacts + i] = cs[i];
  if (joint_rows) {
    float* rows = tab + body_table_floats(M.nc);
    for (int i = lane; i < M.nb * 27; i += 64) rows[(i / 27) * kPRow + i % 27] = M.P[i / 27][i % 27];
  }
  wave_sync();
  if (I && I->cost_kind == 1)
    for (int ci = lane; ci < M.nc; ci += 64) {
      float* ct = tab + kTabContacts + ci * kCt;
      ct[3] = I->f0z[__float_as_int(ct[4])];
    }
  if (I && I->spline_mode == 1 && lane == 0) natural_cubic_diagonal(I->K, tab + kTabSpline);
  wave_sync();
}
__device__ __forceinline__ float contact_point(const float* r, const float* R, const float* p, const float* v,
                                               const float* beta, const float* Rb, const float* pb, const float* agl,
                                               float dt, const ContactLaw& law, float* IA, float* pA, float* vw,
                                               float* fw) {
  const float r0 = r[0], r1 = r[1], r2 = r[2];
  float x[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) x[q] = R[q * 3 + 0] * r0 + R[q * 3 + 1] * r1 + R[q * 3 + 2] * r2;
  float wx[3];
  cross3(v, x, wx);
  const float vB[3] = {v[3] + wx[0], v[4] + wx[1], v[5] + wx[2]};
  const float xB[3] = {p[0] + x[0], p[1] + x[1], p[2] + x[2]};
  float pw[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    pw[q] = pb[q] + Rb[q * 3 + 0] * xB[0] + Rb[q * 3 + 1] * xB[1] + Rb[q * 3 + 2] * xB[2];
    vw[q] = Rb[q * 3 + 0] * vB[0] + Rb[q * 3 + 1] * vB[1] + Rb[q * 3 + 2] * vB[2];
  }
  float fn = 0.f;
  if (pw[2] < 0.f) fn = fmaxf(0.f, -law.k * pw[2] - law.d * vw[2]);
  const float n2 = vw[0] * vw[0] + vw[1] * vw[1] + law.eps * law.eps;
  const float inv_nrm = rsq(n2);
  const float mfn = law.mu * fn * inv_nrm;
  fw[0] = -mfn * vw[0]; fw[1] = -mfn * vw[1]; fw[2] = fn;
  float fB[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) fB[q] = Rb[0 * 3 + q] * fw[0] + Rb[1 * 3 + q] * fw[1] + Rb[2 * 3 + q] * fw[2];
  float xf[3];
  cross3(x, fB, xf);
  pA[0] -= xf[0]; pA[1] -= xf[1]; pA[2] -= xf[2];
  pA[3] -= fB[0]; pA[4] -= fB[1]; pA[5] -= fB[2];
  if (fn > 0.f) {
    // Velocity Jacobian of the contact law (world), tangential-normal coupling
    // dropped: D_w = a I + (d - a) z z^T - a w w^T with a = mu f_n / n and
    // w = v_t / n.  In B axes z -> zb (third row of Rb) and w -> ub = Rb^T w.
    const float aa = mfn;
    const float al = law.d - aa;
    const float zb[3] = {Rb[6], Rb[7], Rb[8]};
    const float wt[2] = {vw[0] * inv_nrm, vw[1] * inv_nrm};
    const float ub[3] = {Rb[0] * wt[0] + Rb[3] * wt[1], Rb[1] * wt[0] + Rb[4] * wt[1], Rb[2] * wt[0] + Rb[5] * wt[1]};
    // added inertia dt P^T D P with P = [-x^x, 1]: with P^T zb = (x x zb, zb) = y1 and
    // P^T ub = (x x ub, ub) = y2 it is dt (al y1 y1^T - a y2 y2^T + a P^T P), where
    // P^T P has blocks |x|^2 I - x x^T, x^x and I
    float w1[3], w2[3];
    cross3(x, zb, w1);
    cross3(x, ub, w2);
    const float x2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    const float dta = dt * aa, dtal = dt * al;
    const float y1[6] = {w1[0], w1[1], w1[2], zb[0], zb[1], zb[2]};
    const float y2[6] = {w2[0], w2[1], w2[2], ub[0], ub[1], ub[2]};
    float t1[6], t2[6];
#pragma unroll
    for (int r = 0; r < 6; ++r) { t1[r] = dtal * y1[r]; t2[r] = dta * y2[r]; }
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int cc = r; cc < 6; ++cc) IA[SI(r, cc)] += t1[r] * y1[cc] - t2[r] * y2[cc];
    const float dax[3] = {dta * x[0], dta * x[1], dta * x[2]};
    const float dx2 = dta * x2;
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int cc = q; cc < 3; ++cc) IA[SI(q, cc)] += (q == cc ? dx2 : 0.f) - dax[q] * x[cc];
    // dt a x^x in the top-right block, dt a I in the bottom-right block
    IA[SI(0, 4)] -= dax[2]; IA[SI(0, 5)] += dax[1];
    IA[SI(1, 3)] += dax[2]; IA[SI(1, 5)] -= dax[0];
    IA[SI(2, 3)] -= dax[1]; IA[SI(2, 4)] += dax[0];
    IA[SI(3, 3)] += dta; IA[SI(4, 4)] += dta; IA[SI(5, 5)] += dta;
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
    for (int q = 0; q < 3; ++q) Dw3[q] = aa * w3[q] + al * zw * zb[q] - aa * uw * ub[q];
    float xd[3];
    cross3(x, Dw3, xd);
    pA[0] += dt * xd[0]; pA[1] += dt * xd[1]; pA[2] += dt * xd[2];
    pA[3] += dt * Dw3[0]; pA[4] += dt * Dw3[1]; pA[5] += dt * Dw3[2];
  }
  return fn;
}

// running-cost terms of one contact point (Sec. IV-A)
__device__ __forceinline__ void contact_cost(const StepConst& sc, float fn, const float* vw, const float* fw, float f0z,
                                             float& lane_cost) {
  if (fn > 0.f) lane_cost += sc.w_cv * (fabsf(vw[0]) + fabsf(vw[1]) + fabsf(vw[2]));
  lane_cost += sc.w_cf * (fabsf(fw[0]) + fabsf(fw[1]) + fabsf(fw[2] - f0z));
}

// end-effector height error: world z of the point ee_pos on a body (R, p) minus z_des
__device__ __forceinline__ float ee_height_error(const float* R, const float* p, const float* ee_pos, const float* Rb,
                                                 const float* pb, float z_des) {
  float xe[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) xe[r] = p[r] + R[r * 3 + 0] * ee_pos[0] + R[r * 3 + 1] * ee_pos[1] + R[r * 3 + 2] * ee_pos[2];
  return pb[2] + Rb[6] * xe[0] + Rb[7] * xe[1] + Rb[8] * xe[2] - z_des;
}

// atan2(y, x) for y, x >= 0: t = min / max in [0, 1], reduced to |u| <= tan(pi/12)
// by atan t = pi/6 + atan((sqrt(3) t - 1) / (t + sqrt(3))) where t > tan(pi/12),
// then the Taylor series of atan u to the u^13 term (truncation below 2e-10);
// atan2 = pi/2 - atan t when y > x.
__device__ __forceinline__ float atan2_pos(float y, float x) {
  const float hi = fmaxf(y, x), lo = fminf(y, x);
  const float t = hi > 0.f ? lo * rcp(hi) : 0.f;
  const float kTan15 = 0.267949192f, kSqrt3 = 1.73205081f;
  const bool big = t > kTan15;
  const float u = big ? (kSqrt3 * t - 1.f) * rcp(t + kSqrt3) : t;
  const float u2 = u * u;
  float sr = 1.f / 13.f;
  sr = fmaf(sr, u2, -1.f / 11.f);
  sr = fmaf(sr, u2, 1.f / 9.f);
  sr = fmaf(sr, u2, -1.f / 7.f);
  sr = fmaf(sr, u2, 1.f / 5.f);
  sr = fmaf(sr, u2, -1.f / 3.f);
  float a = fmaf(sr * u2, u, u);
  if (big) a += 0.523598776f;  // pi/6
  return y > x ? 1.57079633f - a : a;
}

// running-cost terms of the floating base (Sec. IV-A): height error and the
// squared rotation angle between the base and the task's orientation target
// (the identity unless a target is set).
__device__ __forceinline__ float base_cost_term(const StepConst& sc, const float* bq) {
  // orientation residual: rotation angle of R_base^T R_des, i.e. of conj(q_base) q_des
  const float* qt = bq + 3;
  float r0 = qt[0], r1 = qt[1], r2 = qt[2], r3 = qt[3];
  if (sc.or_target) {
    const float d0 = sc.q_des[0], d1 = sc.q_des[1], d2 = sc.q_des[2], d3 = sc.q_des[3];
    r0 = qt[0] * d0 + qt[1] * d1 + qt[2] * d2 + qt[3] * d3;
    r1 = qt[0] * d1 - qt[1] * d0 - qt[2] * d3 + qt[3] * d2;
    r2 = qt[0] * d2 + qt[1] * d3 - qt[2] * d0 - qt[3] * d1;
    r3 = qt[0] * d3 - qt[1] * d2 + qt[2] * d1 - qt[3] * d0;
  }
  const float vn2 = r1 * r1 + r2 * r2 + r3 * r3;
  const float vn = vn2 > 0.f ? vn2 * rsq(vn2) : 0.f;
  const float phi = 2.f * atan2_pos(vn, fabsf(r0));
  return sc.w_h * fabsf(bq[2] - sc.z_des) + sc.w_or * phi * phi;
}

// running-cost terms of a body other than its contacts (Sec. IV-A; effort and
// end-effector terms of the planar-chain task); base_term from base_cost_term
__device__ __forceinline__ void body_cost(const StepConst& sc, int b, bool is_base, bool is_joint, float base_term,
                                          float q, float q0, float tau, const float* R, const float* p,
                                          const float* Rb, const float* pb, float& lane_cost) {
  if (sc.cost_kind == 1) {
    if (is_base) lane_cost += base_term;
    if (is_joint) {
      const float eq = q - q0;
      lane_cost += sc.w_q * eq * eq + sc.w_eff * tau * tau;
    }
  } else {
    if (is_joint) lane_cost += sc.w_tau * tau * tau;
    if (b == sc.ee_body) {
      const float dz = ee_height_error(R, p, sc.ee_pos, Rb, pb, sc.z_des);
      lane_cost += sc.w_ee * dz * dz;
    }
  }
}

// Articulated-body step of a revolute joint (Featherstone's ABA pass 2 in the
// base-axes, own-origin frames): from the body's articulated inertia IA and
// bias pA (children already added) computes U = IA S, 1/D, u and the inertia
// and bias (Ip, pp) carried to the parent's origin.  D includes the armature and
// the implicit PD gain.
__device__ __forceinline__ void backward_joint(const float* IA, const float* pA, const float* ax, const float* c,
                                               const float* e, float tau, float arm, float gain, float* U,
                                               float& invD, float& u, float* Ip, float* pp) {
  // S = (ax, 0): U = IA S, D = S.U + g, u = tau - S.pA
#pragma unroll
  for (int r = 0; r < 6; ++r) U[r] = IA[SI(r, 0)] * ax[0] + IA[SI(r, 1)] * ax[1] + IA[SI(r, 2)] * ax[2];
  const float Dv = (arm + gain) + (ax[0] * U[0] + ax[1] * U[1] + ax[2] * U[2]);
  invD = rcp(Dv);
  u = tau - (ax[0] * pA[0] + ax[1] * pA[1] + ax[2] * pA[2]);
  // Ia = IA - U U^T / D, with W = U / D
  float W[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) W[r] = U[r] * invD;
  float Ia[21];
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int cc = r; cc < 6; ++cc) Ia[SI(r, cc)] = IA[SI(r, cc)] - U[r] * W[cc];
  float Iac[6];
  sym6_mv(Ia, c, Iac);
  const float uD = u * invD;
  float pa[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) pa[q] = pA[q] + Iac[q] + U[q] * uD;
  shift_inertia_to_parent(Ia, e, Ip);
  float ef[3];
  cross3(e, pa + 3, ef);
  pp[0] = pa[0] + ef[0]; pp[1] = pa[1] + ef[1]; pp[2] = pa[2] + ef[2];
  pp[3] = pa[3]; pp[4] = pa[4]; pp[5] = pa[5];
}

// Floating-base root: solves IA0 a0' = -pA0 by Cholesky (a0' = a0 - a_g).
__device__ __forceinline__ void base_solve(const float* IA, const float* pA, float* a0) {
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
  float y[6];
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
}

// ABA pass 3 for a revolute joint: parent acceleration al (gravity-offset, about
// the parent origin) -> joint acceleration qdd and the body's own a'.
__device__ __forceinline__ float forward_joint(const float* al, const float* e, const float* c, const float* U, float u,
                                               float invD, const float* ax, float* aout) {
  float a[6];
  shift_motion(al, e, a);
#pragma unroll
  for (int q = 0; q < 6; ++q) a[q] += c[q];
  float Ua = 0.f;
#pragma unroll
  for (int q = 0; q < 6; ++q) Ua = fmaf(U[q], a[q], Ua);
  const float qdd = (u - Ua) * invD;
  aout[0] = a[0] + ax[0] * qdd; aout[1] = a[1] + ax[1] * qdd; aout[2] = a[2] + ax[2] * qdd;
  aout[3] = a[3]; aout[4] = a[4]; aout[5] = a[5];
  return qdd;
}

// ---------------------------------------------------------------------------
// Body schedule: one lane per body, the tree swept level by level through LDS.
// terminal = true evaluates only the kinematics and the end-effector height term
// of the terminal cost (end-effector task) at the current state.
// ---------------------------------------------------------------------------
// D > 0: the tree is at most D levels deep, fixed at compile time so the level
// loops unroll (levels below the tree have no body and cost only their shifts).
// Unroll counts of the loops over levels 1..D and D..0 (1: a run-time loop).
// A body's kinematics in a physics step (base axes, about the body origin):
// rotation R, origin p, lever arm e from the parent origin, joint axis ax,
// twist v, velocity product c and bias acceleration beta.  The base's R, p and
// beta are the identity frame and zero (base_frame).  The legged-tree kernels
// keep it across steps (set once by init_kin): a lane whose frame a neighbour
// reads before the lane's own level then hands over its previous step's
// values, which the neighbour does not use (the compiler would otherwise
// materialise the not-yet-computed values); the other kernels, with less
// register room, take it fresh every step.
struct BodyKin {
  float R[9], p[3], e[3], ax[3], v[6], c[6], beta[6];
};
__device__ __forceinline__ void base_frame(BodyKin& k) {
#pragma unroll
  for (int i = 0; i < 9; ++i) k.R[i] = (i % 4 == 0) ? 1.f : 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) k.p[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 6; ++i) k.beta[i] = 0.f;
}
__device__ __forceinline__ void init_kin(BodyKin& k) {
  base_frame(k);
#pragma unroll
  for (int i = 0; i < 3; ++i) k.e[i] = k.ax[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 6; ++i) k.v[i] = k.c[i] = 0.f;
}

template <int D> constexpr int kLevelUnroll = D > 0 ? D : 1;
template <int D> constexpr int kLevelUnrollRoot = D > 0 ? D + 1 : 1;

// LEG = 1: the tree is a floating base with serial chains hanging off it
// (every joint body's parent is the previous lane, or the base for a chain's
// first body; no body but the base has more than one child), so a frame, an
// acceleration or a carried inertia always comes from the neighbouring lane
// except the base's, which gathers the chains through LDS.  LEG = 2: such a
// tree with four chains of three bodies in groups of 16 lanes (the chains'
// first bodies at lanes 1, 4, 7 and 10), whose base gathers the chains by row
// shifts instead.  LEG = 3: a fixed-base serial chain (body b's parent is body
// b - 1, the first body's the world), so every hand-over is a neighbour's and
// nothing goes through LDS.  The same arithmetic as the general form (children
// added in the same order), with its LDS paths and their branches compiled out.
template <int G, int D = 0, int LEG = 0>
__device__ void physics_step(const StepConst& sc, const BodyConst& bc, const float* tab, float* __restrict__ gs,
                             int b, bool body_lane, StepIO& io, BodyKin& kin_kept, bool want_cost,
                             bool terminal = false) {
  const int maxd = D > 0 ? D : sc.max_depth;
  // the joint-rotation constants are read first so the LDS latency passes
  // under the PD law, the base cost and frame B
  float Pt[28];
  load_rotation_constants(bc.P, Pt);
  float* slots = gs;
  const int fb = LEG == 3 ? 0 : (LEG != 0 ? 1 : sc.fb);  // legged trees have a floating base, serial chains not
  const bool is_base = body_lane && fb && b == 0;
  const bool is_joint = body_lane && !is_base;

  float tau = 0.f, gain = 0.f;
  if (is_joint) pd_law(bc.kp, bc.kd, bc.taumax, io.dt, io.q, io.v, io.qref, io.vref, tau, gain);
  io.tau = tau;
  float base_term = 0.f;
  if (want_cost && is_base && sc.cost_kind == 1) base_term = base_cost_term(sc, io.bq);

  // ---- frame B: world pose of the base.  Every lane carries the base state
  //      (position, quaternion, twist), so every lane forms it in registers.
  float* Rb = io.Rb;
  float pb[3];
  if (fb) {
    quat_R(io.bq + 3, Rb);
    pb[0] = io.bq[0]; pb[1] = io.bq[1]; pb[2] = io.bq[2];
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Rb[k] = (k % 4 == 0) ? 1.f : 0.f;
    pb[0] = pb[1] = pb[2] = 0.f;
  }

  // ---- forward kinematics, level by level (slot: R, p, v, beta about the body origin)
  BodyKin kin_step;  // the other kernels: fresh every step
  BodyKin& kin = LEG != 0 ? kin_kept : kin_step;
  float(&R)[9] = kin.R;
  float(&p)[3] = kin.p;
  float(&e)[3] = kin.e;
  float(&ax)[3] = kin.ax;
  float(&v)[6] = kin.v;
  float(&c)[6] = kin.c;
  float(&beta)[6] = kin.beta;
  const int depth = bc.depth;
  if (is_base) {  // (lever arm, axis and velocity product are never read for the base)
    if constexpr (LEG == 0) base_frame(kin);
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = io.bv[k];
  }
  float C[9];
  if (is_joint) {
    float cq, sq;
    sincosf(io.q, &sq, &cq);
    joint_rotation_of(Pt, cq, sq, C);
  }
#pragma unroll kLevelUnroll<D>
  for (int d = 1; d <= maxd; ++d) {
    float sR[9], sp[3], sv[6], sb[6];  // the previous lane's frame (level d - 1)
    if (d > 1) {
#pragma unroll
      for (int k = 0; k < 9; ++k) sR[k] = from_prev_lane(R[k]);
#pragma unroll
      for (int k = 0; k < 3; ++k) sp[k] = from_prev_lane(p[k]);
#pragma unroll
      for (int k = 0; k < 6; ++k) { sv[k] = from_prev_lane(v[k]); sb[k] = from_prev_lane(beta[k]); }
    }
    if (is_joint && depth == d) {
      const int lam = bc.parent;
      if (fb && d == 1) {  // a child of the floating base: frame identity, twist bv
        fk_base_child(io.bv, C, bc.p_tree, bc.axis_p, io.v, R, p, e, ax, v, c, beta);
      } else {
        float Rl[9], pl[3], vl[6], bl[6];
        if (LEG == 3 ? d > 1 : (LEG != 0 || (bc.flags & kAdjParent))) {
#pragma unroll
          for (int k = 0; k < 9; ++k) Rl[k] = sR[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) pl[k] = sp[k];
#pragma unroll
          for (int k = 0; k < 6; ++k) { vl[k] = sv[k]; bl[k] = sb[k]; }
        } else if (LEG != 3 && lam >= 0) {
          get_frame(slots + lam * kSlot, Rl, pl, vl, bl);
        } else {
#pragma unroll
          for (int k = 0; k < 9; ++k) Rl[k] = (k % 4 == 0) ? 1.f : 0.f;
#pragma unroll
          for (int k = 0; k < 3; ++k) pl[k] = 0.f;
#pragma unroll
          for (int k = 0; k < 6; ++k) { vl[k] = 0.f; bl[k] = 0.f; }
        }
        fk_joint(Rl, pl, vl, bl, C, bc.p_tree, bc.axis_p, io.v, R, p, e, ax, v, c, beta);
      }
      if (LEG == 0 && (bc.flags & kFrameOut)) put_frame(slots + b * kSlot, R, p, v, beta);
    }
    wave_sync();
  }

  // ---- rigid-body inertia, bias force, contacts (all body lanes in parallel)
  float IA[21], pA[6];
  float lane_cost = 0.f;
  uint32_t mask = 0u;
  if (terminal) {
    if (body_lane && sc.cost_kind == 0 && b == sc.ee_body) {
      const float dz = ee_height_error(R, p, sc.ee_pos, Rb, pb, sc.z_des);
      lane_cost = sc.w_ee * dz * dz;
    }
    io.cost = lane_cost;
    io.mask = 0u;
    wave_sync();
    return;
  }
  const float g = sc.g;
  // gravity as a spatial acceleration in B axes: (0, Rb^T (0, 0, -g)), the same about any origin
  const float agl[3] = {-g * Rb[6], -g * Rb[7], -g * Rb[8]};
  if (body_lane) {
    // every body's rigid inertia about its origin, the base's too (its frame is
    // the identity: every schedule forms it from the same constants the same way)
    body_inertia(R, bc.com, bc.Ic, bc.mass, IA);
    bias_force(IA, v, pA);

    // contacts carried by this body (point x relative to the body origin); the
    // first one's row is held in registers, further ones are read from the table
    // (LEG = 2: at most one contact per body, so no loop; the depth-6 kernels read
    // the first row from the table too, and spend the registers on the layout
    // hints of rollout_item)
    const int c0 = bc.c_begin, cn = LEG == 2 ? min(bc.c_count, 1) : bc.c_count;
    for (int ci = c0; ci < c0 + cn; ++ci) {
      float ct[5];
      if (ci == c0 && D != 6) {
#pragma unroll
        for (int k = 0; k < 5; ++k) ct[k] = bc.ct0[k];
      } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) ct[k] = tab[kTabContacts + ci * kCt + k];
      }
      float vw[3], fw[3];
      const float fn = contact_point(ct, R, p, v, beta, Rb, pb, agl, io.dt, sc.law, IA, pA, vw, fw);
      if (fn > 0.f) mask |= 1u << __float_as_int(ct[4]);
      if (want_cost && sc.cost_kind == 1) contact_cost(sc, fn, vw, fw, ct[3], lane_cost);
    }
    if (want_cost) body_cost(sc, b, is_base, is_joint, base_term, io.q, bc.q0, tau, R, p, Rb, pb, lane_cost);
  }
  io.cost = lane_cost;
  io.mask = mask;
  wave_sync();

  // ---- backward sweep, leaves to root: each joint lane publishes its
  //      articulated inertia and bias already carried to its parent's origin
  float U[6], invD = 0.f, u = 0.f;
  // kFoldAll (depth-specialised kernels): the inertia and bias carried to the
  // parent are zero until the lane's own level, then its body's (kept for the
  // rest of the sweep), and every lane adds its next lane's after each level.
  // The run-time-depth kernel keeps them per level (unset on lanes of other
  // levels) and adds them on the parents only.
  constexpr bool kFoldAll = D > 0;
  float Ip[21], pp[6];
  if constexpr (kFoldAll) {
#pragma unroll
    for (int q = 0; q < 21; ++q) Ip[q] = 0.f;
#pragma unroll
    for (int q = 0; q < 6; ++q) pp[q] = 0.f;
  }
#pragma unroll kLevelUnrollRoot<D>
  for (int d = maxd; d >= 0; --d) {
    if constexpr (LEG == 2) {
      if (d == 0) {
        // the base adds chains 2, 3 and 4 (lanes 4, 7 and 10 of the group) in
        // child order; every lane adds, only the base's sums are used (the
        // joint lanes' articulated inertias are no longer needed)
#pragma unroll
        for (int q = 0; q < 21; ++q) IA[q] += from_row_lane<4>(Ip[q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) pA[q] += from_row_lane<4>(pp[q]);
#pragma unroll
        for (int q = 0; q < 21; ++q) IA[q] += from_row_lane<7>(Ip[q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) pA[q] += from_row_lane<7>(pp[q]);
#pragma unroll
        for (int q = 0; q < 21; ++q) IA[q] += from_row_lane<10>(Ip[q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) pA[q] += from_row_lane<10>(pp[q]);
      }
    }
    if (body_lane && depth == d) {
      const int nch = bc.n_child;
      if (LEG != 2 && LEG != 3 && (LEG == 0 || d == 0) && nch > 0) {
        // children reached through LDS: the first kFold records are read together
        // (a missing child reads this lane's own slot and is not added), then
        // added in child order; more children follow one by one
        constexpr int kFold = (D > 0 && D != 6) ? 3 : 2;  // (the generic and depth-6 kernels have fewer registers to spare)
        float t[kFold][28];
#pragma unroll
        for (int k = 0; k < kFold; ++k) {
          const float* src = slots + (k < nch ? child_of(bc, k) : b) * kSlot;
#pragma unroll
          for (int q = 0; q < 7; ++q) {
            const float4 x = get4(src + 4 * q);
            t[k][4 * q] = x.x; t[k][4 * q + 1] = x.y; t[k][4 * q + 2] = x.z; t[k][4 * q + 3] = x.w;
          }
        }
#pragma unroll
        for (int k = 0; k < kFold; ++k)
          if (k < nch) {
#pragma unroll
            for (int q = 0; q < 21; ++q) IA[q] += t[k][q];
#pragma unroll
            for (int q = 0; q < 6; ++q) pA[q] += t[k][21 + q];
          }
#pragma unroll 1
        for (int k = kFold; k < nch; ++k) add_art(slots + child_of(bc, k) * kSlot, IA, pA);
      }
      if (is_joint) {
        backward_joint(IA, pA, ax, c, e, tau, bc.arm, gain, U, invD, u, Ip, pp);
        if (LEG != 2 && LEG != 3 && (LEG == 0 || d == 1) && (bc.flags & kArtOut)) put_art(slots + b * kSlot, Ip, pp);
      }
    }
    wave_sync();
    if (d > 0) {
      // a parent at level d - 1 adds its first child's contribution first, then
      // the others'
      if constexpr (kFoldAll) {
        // every lane adds its next lane's carried inertia (one DPP add): in a
        // depth-first numbering the next body is this body's child iff it is
        // one level deeper, so a lane of level d - 1 takes its first child's; a
        // lane not yet swept takes a zero (its next lane is not swept yet
        // either); a lane already swept no longer needs its sums
#pragma unroll
        for (int q = 0; q < 21; ++q) IA[q] += from_next_lane(Ip[q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) pA[q] += from_next_lane(pp[q]);
      } else {
        float sI[21], spp[6];
#pragma unroll
        for (int q = 0; q < 21; ++q) sI[q] = from_next_lane(Ip[q]);
#pragma unroll
        for (int q = 0; q < 6; ++q) spp[q] = from_next_lane(pp[q]);
        if (body_lane && depth == d - 1 && (bc.flags & kAdjChild)) {
#pragma unroll
          for (int q = 0; q < 21; ++q) IA[q] += sI[q];
#pragma unroll
          for (int q = 0; q < 6; ++q) pA[q] += spp[q];
        }
      }
    }
  }

  // ---- root: floating base solves IA0 a0' = -pA0 (Cholesky); fixed roots use -a_g
  float a0[6];  // the base's a' = a0 - a_g, then in every lane of its rollout
  if (is_base) base_solve(IA, pA, a0);
  if (fb) {
#pragma unroll
    for (int k = 0; k < 6; ++k) a0[k] = from_group_lane0<G>(a0[k]);
    io.ba[0] = a0[0]; io.ba[1] = a0[1]; io.ba[2] = a0[2];
    io.ba[3] = a0[3] + agl[0]; io.ba[4] = a0[4] + agl[1]; io.ba[5] = a0[5] + agl[2];
  }

  // ---- forward sweep: accelerations, root to leaves
  float qdd = 0.f;
  float a[6], sa[6];  // this lane's and the previous lane's acceleration
#pragma unroll kLevelUnroll<D>
  for (int d = 1; d <= maxd; ++d) {
    if (is_joint && depth == d) {
      const int lam = bc.parent;
      float al[6];
      if (fb && d == 1) {
#pragma unroll
        for (int k = 0; k < 6; ++k) al[k] = a0[k];
      } else if (LEG == 3 ? d > 1 : (LEG != 0 || (bc.flags & kAdjParent))) {
#pragma unroll
        for (int k = 0; k < 6; ++k) al[k] = sa[k];
      } else if (LEG != 3 && lam >= 0) {
        get_acc(slots + lam * kSlot, al);
      } else {
        // fixed world: a' = -a_g = (0, 0, 0, 0, 0, g); its angular part is zero, so no shift term
        al[0] = al[1] = al[2] = 0.f; al[3] = 0.f; al[4] = 0.f; al[5] = g;
      }
      qdd = forward_joint(al, e, c, U, u, invD, ax, a);
      if (LEG == 0 && (bc.flags & kFrameOut)) put_acc(slots + b * kSlot, a);
    }
    wave_sync();
    if (d < maxd) {
#pragma unroll
      for (int k = 0; k < 6; ++k) sa[k] = from_prev_lane(a[k]);
    }
  }
  io.qdd = qdd;
}

// ---------------------------------------------------------------------------
// Knot sampling for one rollout group: counter-based normals, perturbation,
// position clip and bound-aware velocity clamp.
// ---------------------------------------------------------------------------
// Sample n's position and velocity knot of one element (Alg. 1 sampling step:
// the nominal (nq, nv) perturbed by the iteration's std sq at the element's
// knot, the position clipped to the joint range [lo, hi], the velocity clamped
// by eq. vel-clamp) from the uniform words (xa, xb) of its counter-based block,
// by Box-Muller.  Sample 0 is the nominal itself (clipped and clamped the same
// way).  The rollout's sampler and the update's regeneration both call this, so
// they give the same bits.
struct ElemConst {
  float sq, lo, hi;  // std at the element's knot, joint range
  int m;             // element index k nu + jj
};
__device__ __forceinline__ ElemConst elem_const(const DevModel& M, const DevInst& I, const float* sig, int m) {
  const int k = m / I.nu, jj = m % I.nu;
  return ElemConst{sig[k], M.qmin[jj], M.qmax[jj], m};
}
__device__ __forceinline__ void perturb_element(const ElemConst& ec, float delta, float nq, float nv, int n,
                                                uint32_t xa, uint32_t xb, bool with_velocity, float& tq,
                                                float& tv) {
  float zq = 0.f, zv = 0.f;
  if (n > 0) {
    const float ua = u01(xa), ub = u01(xb);
    const float r = sqrtf(-2.f * logf(ua));
    zq = r * cospif(2.f * ub);
    zv = r * sinpif(2.f * ub);
  }
  tq = fminf(fmaxf(fmaf(ec.sq, zq, nq), ec.lo), ec.hi);
  tv = 0.f;
  if (with_velocity) {
    const float sv = ec.sq / delta;
    const float lim = 2.f * fminf(ec.hi - tq, tq - ec.lo) / delta;
    tv = fminf(fmaxf(fmaf(sv, zv, nv), -lim), lim);
  }
}

// The counter-based block blk of sample n in iteration I.iter at tick `tick`
// (key = seed; counter = (blk, n, iter, tick)); sample 0 draws none.
__device__ __forceinline__ uint4 sample_words(const DevInst& I, int n, int blk, uint32_t tick) {
  if (n == 0) return make_uint4(0u, 0u, 0u, 0u);
  return philox(make_uint4((uint32_t)blk, (uint32_t)n, (uint32_t)I.iter, tick), make_uint2(I.seed_lo, I.seed_hi));
}
__device__ __forceinline__ uint32_t sample_tick(const DevInst& I) {
  return I.use_tick_value ? I.tick_value : *I.tick_ptr;
}

// Knot sampling for one rollout group: block blk gives elements 2 blk and
// 2 blk + 1 (its words x, y and z, w); the lanes of the group take the blocks
// in turn.
template <int G>
__device__ void sample_group(const DevModel& M, const DevInst& I, int n, int l, float* knots, bool valid,
                             const float* tab, const float* nominal = nullptr) {
  const float* nom = nominal ? nominal : I.nominal;
  const int K = I.K, nu = I.nu, KU = K * nu;
  const int nblk = (KU + 1) / 2;
  const float* sig = I.sigma + I.iter * K;
  const uint32_t tick = sample_tick(I);
  const bool store = valid && I.store_samples;
  const bool with_v = I.spline_mode == 0;
  for (int blk = l; blk < nblk; blk += G) {
    const uint4 x = sample_words(I, n, blk, tick);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int m = 2 * blk + half;
      if (m >= KU) break;
      float tq, tv;
      perturb_element(elem_const(M, I, sig, m), I.delta, nom[m], with_v ? nom[KU + m] : 0.f, n,
                      half ? x.z : x.x, half ? x.w : x.y, with_v, tq, tv);
      knots[m] = tq;
      if (store) I.samples[(size_t)n * I.E + m] = tq;
      if (with_v) {
        knots[KU + m] = tv;
        if (store) I.samples[(size_t)n * I.E + KU + m] = tv;
      }
    }
  }
  if (I.spline_mode != 0) {
    // position-only variants: knot slopes of the spline through the sampled positions
    wave_sync();
    for (int jj = l; jj < nu; jj += G) {
      position_spline_slopes(I.spline_mode, K, nu, jj, I.delta, tab + kTabSpline, knots);
      if (store)
        for (int k = 0; k < K; ++k) I.samples[(size_t)n * I.E + KU + k * nu + jj] = knots[KU + k * nu + jj];
    }
  }
}

// Hermite reference of joint jj (eq. hermite_segment and its time derivative).
// The knots of one segment, slopes scaled by the knot spacing delta, are loaded
// once per segment; the curve is then evaluated at local time s in [0, 1].
struct HermiteSeg {
  float q0, q1, m0, m1;
};
__device__ __forceinline__ HermiteSeg hermite_segment(const float* knots, int K, int nu, int seg, int jj, float delta) {
  const int KU = K * nu;
  HermiteSeg h;
  h.q0 = knots[seg * nu + jj];
  h.q1 = knots[(seg + 1) * nu + jj];
  h.m0 = delta * knots[KU + seg * nu + jj];
  h.m1 = delta * knots[KU + (seg + 1) * nu + jj];
  return h;
}
__device__ __forceinline__ void hermite_eval(const HermiteSeg& h, float s, float inv_delta, float* qr, float* vr) {
  const float s2 = s * s, s3 = s2 * s;
  const float h00 = 2.f * s3 - 3.f * s2 + 1.f, h10 = s3 - 2.f * s2 + s, h01 = -2.f * s3 + 3.f * s2, h11 = s3 - s2;
  const float d00 = 6.f * s2 - 6.f * s, d10 = 3.f * s2 - 4.f * s + 1.f, d01 = -6.f * s2 + 6.f * s, d11 = 3.f * s2 - 2.f * s;
  *qr = h00 * h.q0 + h10 * h.m0 + h01 * h.q1 + h11 * h.m1;
  *vr = (d00 * h.q0 + d10 * h.m0 + d01 * h.q1 + d11 * h.m1) * inv_delta;
}
// At fine step f of F inside a rollout: the segment seg = floor(f (K-1) / F) and
// the remainder rem = f (K-1) - seg F are exact integers kept by the caller
// (StepClock); the local time is s = rem (1/F).
__device__ __forceinline__ void hermite(const float* knots, int K, int nu, float inv_F, float delta, float inv_delta,
                                        int seg, int rem, int jj, float* qr, float* vr) {
  hermite_eval(hermite_segment(knots, K, nu, seg, jj, delta), (float)rem * inv_F, inv_delta, qr, vr);
}

// Fine-step bookkeeping without integer division: the Hermite segment and
// remainder of step f (f (K-1) = seg F + rem, 0 <= rem < F; for f < F the
// segment never exceeds K-2), the substep within a control step and the
// control-step index.
struct StepClock {
  int seg = 0, rem = 0, sub = 0, h = 0;
  template <bool H = false>
  __device__ __forceinline__ void advance(int K, int F, int nsub) {
    rem += K - 1;
    while (MPPI_RARE(H, rem >= F)) {
      rem -= F;
      ++seg;
    }
    if (++sub == nsub) {
      sub = 0;
      ++h;
    }
  }
};

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
// (R: the rotation of the quaternion bq[3..6], as quat_R gives it)
template <bool H = false>
__device__ __forceinline__ void integrate_base_R(float* bq, float* bv, const float* ba, float dt, const float* R) {
#pragma unroll
  for (int k = 0; k < 6; ++k) bv[k] = fmaf(dt, ba[k], bv[k]);
#pragma unroll
  for (int r = 0; r < 3; ++r) bq[r] += dt * (R[r * 3 + 0] * bv[3] + R[r * 3 + 1] * bv[4] + R[r * 3 + 2] * bv[5]);
  const float wn2 = bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2];
  // exp of the half rotation: (cos th, sin th w / |w|), th = |w| dt / 2; below
  // th = 1/4 by the Taylor series of cos th and sin th / th to the th^6 term
  // (truncation below 5e-10, under float rounding), which needs th^2 only
  const float hdt = 0.5f * dt;
  const float t2 = (hdt * hdt) * wn2;
  float e0 = 1.f + t2 * (-0.5f + t2 * (1.f / 24.f + t2 * (-1.f / 720.f)));
  float k = hdt * (1.f + t2 * (-1.f / 6.f + t2 * (1.f / 120.f + t2 * (-1.f / 5040.f))));
  if (MPPI_RARE(H, !(t2 < 0.0625f))) {
    const float wn = sqrtf(wn2);
    float sn, cs;
    sincosf(hdt * wn, &sn, &cs);
    e0 = cs;
    k = sn * rcp(wn);
  }
  const float e1 = k * bv[0], e2 = k * bv[1], e3 = k * bv[2];
  const float a0 = bq[3], a1 = bq[4], a2 = bq[5], a3 = bq[6];
  const float r0 = a0 * e0 - a1 * e1 - a2 * e2 - a3 * e3;
  const float r1 = a0 * e1 + a1 * e0 + a2 * e3 - a3 * e2;
  const float r2 = a0 * e2 - a1 * e3 + a2 * e0 + a3 * e1;
  const float r3 = a0 * e3 + a1 * e2 - a2 * e1 + a3 * e0;
  const float inv = rsq(r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
  bq[3] = r0 * inv; bq[4] = r1 * inv; bq[5] = r2 * inv; bq[6] = r3 * inv;
}
__device__ __forceinline__ void integrate_base(float* bq, float* bv, const float* ba, float dt) {
  float R[9];
  quat_R(bq + 3, R);
  integrate_base_R(bq, bv, ba, dt, R);
}

// ---------------------------------------------------------------------------
// Fused rollout of one work item: 64/G rollouts of one instance, samples
// w.y .. w.y + 64/G - 1 (those >= N are computed but not stored).
// ---------------------------------------------------------------------------
// steps control steps are simulated (the horizon for a rollout).  With state_out
// set (state prediction, one sample) the state reached is written there and
// no cost is formed.
// Per-step record of a traced rollout (verification of the simulate step of
// Alg. 1, step by step): record h < H holds the state (q, v) at the start of
// control step h, the accelerations of its first physics substep, its running
// cost and its contact mask (bits); record H the final state, zero
// accelerations, the terminal cost and 0.  Layout [q | v | qdd | cost | mask].
template <int G>
__device__ __forceinline__ void trace_record(const DevInst& I, int n, bool valid, int h, int fb, int nq, int nv,
                                             bool is_joint, int j, int b, int l, const StepIO& io, bool with_acc,
                                             float cost, uint32_t mk) {
  if (!valid) return;
  const int slot = I.trace_map[n];
  if (slot < 0) return;
  const int rec = nq + 2 * nv + 2;
  float* r = I.trace + ((size_t)slot * (I.H + 1) + h) * rec;
  if (is_joint) {
    r[(fb ? 7 : 0) + j] = io.q;
    r[nq + (fb ? 6 : 0) + j] = io.v;
    r[nq + nv + (fb ? 6 : 0) + j] = with_acc ? io.qdd : 0.f;
  }
  if (fb && b == 0) {
    for (int k = 0; k < 7; ++k) r[k] = io.bq[k];
    for (int k = 0; k < 6; ++k) {
      r[nq + k] = io.bv[k];
      r[nq + nv + k] = with_acc ? io.ba[k] : 0.f;
    }
  }
  if (l == 0) {
    r[nq + 2 * nv] = cost;
    r[nq + 2 * nv + 1] = __uint_as_float(mk);
  }
}

// x0_in / nominal_in (nullable) replace the instance's staged state and nominal.
// TR: also write the per-step records of traced rollouts (verification kernel).
// per_item: called once per work item in a loop (the persistent form): the lane
// index is passed through an empty asm statement that claims to change it, so
// what derives from it (group, body, LDS addresses) is formed again for each
// item instead of being held live across the loop, which would take the kernel
// past the two-wavefront register budget.
template <int G, int D = 0, bool TR = false, int LEG = 0>
__device__ __attribute__((always_inline)) void rollout_item(const DevInst& I, int first, int group_stride,
                                                            int table_floats, float* smem, int steps,
                                                            float* state_out, const float* x0_in = nullptr,
                                                            const float* nominal_in = nullptr, bool per_item = false) {
  const float* x0 = x0_in ? x0_in : I.x0;
  // issue priority among the wavefronts sharing a SIMD (the server raises it for
  // the trees with the longest per-step chains)
  switch (I.wave_prio) {
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    case 3: __builtin_amdgcn_s_setprio(3); break;
    default: break;
  }
  int lane = threadIdx.x;
  if (per_item) asm volatile("" : "+v"(lane));
  const int grp = lane / G, l = lane % G;
  const DevModel& M = *I.model;
  float* tab = smem;
  stage_model_table(M, &I, tab, lane, true);
  const int n = first + grp;
  const bool valid = n < I.N;
  float* gs = smem + table_floats + grp * group_stride;
  float* knots = gs + G * kSlot + 16;
  float* red = knots + ((I.E + 3) & ~3);

  // knots of this sample
  if (I.generate) {
    sample_group<G>(M, I, valid ? n : 0, l, knots, valid, tab, nominal_in);
  } else {
    const float* src = I.samples + (size_t)(valid ? n : 0) * I.E;
    for (int e = l; e < I.E; e += G) knots[e] = src[e];
  }
  wave_sync();

  const StepConst sc = load_step_const(M, &I, 0.f);
  const int fb = LEG == 3 ? 0 : (LEG != 0 ? 1 : sc.fb), nb = M.nb, nq = fb ? 7 + M.nu : M.nu;
  const bool body_lane = l < nb;
  const int b = l;
  const bool is_joint = body_lane && !(fb && b == 0);
  const int j = b - fb;
  StepIO io;
  io.q = io.v = 0.f;
  if (is_joint) {
    io.q = x0[(fb ? 7 : 0) + j];
    io.v = x0[nq + (fb ? 6 : 0) + j];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) io.bq[k] = fb ? x0[k] : 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) io.bv[k] = fb ? x0[nq + k] : 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) io.ba[k] = 0.f;
  io.qref = io.vref = 0.f;
  io.dt = sc.dt;

  BodyConst bc;
  load_body(M, &I, b, body_lane, tab, bc);
  BodyKin kin_kept;  // legged trees: kept across the steps (see BodyKin)
  if constexpr (LEG != 0) init_kin(kin_kept);
  uint32_t* const masks = I.masks;
  const int H = I.H, F = sc.F, F_run = steps * sc.nsub;
  float acc = 0.f;
  StepClock clk;
  // this joint's knots on the current segment, kept in registers across steps
  // where the register budget allows (depth-specialised kernels), else reloaded
  // every step (the same values)
  HermiteSeg hs{0.f, 0.f, 0.f, 0.f};
  int hseg = -1;
  // rare paths laid out of line (MPPI_RARE) where the registers allow it
  constexpr bool kHints = LEG != 0 || D == 6;
  for (int f = 0; f < F_run; ++f) {
    const bool control = clk.sub == 0;
    if (D == 0 || MPPI_RARE(kHints, clk.seg != hseg)) {
      hseg = clk.seg;
      if (is_joint) hs = hermite_segment(knots, sc.K, sc.nu, hseg, j, sc.delta);
    }
    // (lanes without a joint evaluate zero knots and never use the result)
    hermite_eval(hs, (float)clk.rem * sc.inv_F, sc.inv_delta, &io.qref, &io.vref);
    if (sc.spline_mode != 0) io.vref = 0.f;  // position-only variants: zero velocity targets
    physics_step<G, D, LEG>(sc, bc, tab, gs, b, body_lane, io, kin_kept, control);
    if (control) {
      acc += io.cost;
      if (MPPI_RARE(kHints, masks != nullptr)) {
        const uint32_t mk = group_or<G>(io.mask, red, l);
        if (l == 0 && valid) masks[(size_t)n * H + clk.h] = mk;
        if (TR && I.trace) {
          const float c = group_sum<G>(io.cost, red, l);
          trace_record<G>(I, n, valid, clk.h, fb, nq, nq - fb, is_joint, j, b, l, io, true, c, mk);
        }
      }
    }
    // joints (other lanes hold q = qd = qdd = 0)
    io.v = fmaf(io.dt, io.qdd, io.v);
    io.q = fmaf(io.dt, io.v, io.q);
    if (fb) integrate_base_R<kHints>(io.bq, io.bv, io.ba, io.dt, io.Rb);  // every lane: the same base state
    clk.advance<kHints>(sc.K, F, sc.nsub);
  }
  if (state_out) {
    if (valid) {
      if (is_joint) {
        state_out[(fb ? 7 : 0) + j] = io.q;
        state_out[nq + (fb ? 6 : 0) + j] = io.v;
      }
      if (fb && b == 0) {
#pragma unroll
        for (int k = 0; k < 7; ++k) state_out[k] = io.bq[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) state_out[nq + k] = io.bv[k];
      }
    }
    return;
  }

  // terminal cost
  float term_e = 0.f;
  if (sc.cost_kind == 1) {
    if (fb && b == 0) {
      const float T = (float)H * I.dt;
      float e = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float target = (k == 2 && I.targets->terminal_z_abs) ? I.targets->z_terminal : x0[k] + I.targets->v_des[k] * T;
        e += fabsf(io.bq[k] - target);
      }
      acc += I.w_H * e;
      term_e = e;
    }
  } else {
    // end-effector height at x_H
    physics_step<G, D, LEG>(sc, bc, tab, gs, b, body_lane, io, kin_kept, false, true);
    acc += io.cost;
  }
  if (TR && masks && I.trace) {
    const float ct = group_sum<G>(sc.cost_kind == 1 ? I.w_H * term_e : io.cost, red, l);
    trace_record<G>(I, n, valid, H, fb, nq, nq - fb, is_joint, j, b, l, io, false, ct, 0u);
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
// D > 0: every instance of the launch is at most D levels deep.
// x0_in / nominal_in (nullable, one instance only): the state and the nominal
// to use instead of the instance's staged copies.
// LEG: every instance of the launch is a legged tree of that kind (see physics_step).
template <int G, int D, int LEG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void rollout_kernel(
    const DevInst* __restrict__ insts, const int2* __restrict__ work, int group_stride, int table_floats,
    const float* __restrict__ x0_in, const float* __restrict__ nominal_in) {
  extern __shared__ float smem[];
  constexpr int R = 64 / G;
  const int2 w = work ? work[blockIdx.x] : make_int2(0, (int)blockIdx.x * R);
  const DevInst& I = insts[w.x];
  rollout_item<G, D, false, LEG>(I, w.y, group_stride, table_floats, smem, I.H, nullptr, x0_in, nominal_in);
}

// The rollout kernel with per-step records of the traced rollouts (same launch
// shape and arithmetic; verification only).
template <int G, int D, int LEG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void rollout_trace_kernel(
    const DevInst* __restrict__ insts, const int2* __restrict__ work, int group_stride, int table_floats) {
  extern __shared__ float smem[];
  constexpr int R = 64 / G;
  const int2 w = work ? work[blockIdx.x] : make_int2(0, (int)blockIdx.x * R);
  const DevInst& I = insts[w.x];
  rollout_item<G, D, true, LEG>(I, w.y, group_stride, table_floats, smem, I.H, nullptr);
}

// State prediction: sample 0 of the instance (its knots read from samples) run
// for `steps` control steps from x0; the state reached goes to state_out.
template <int G>
__global__ __launch_bounds__(64) void predict_kernel(const DevInst* __restrict__ inst, int steps,
                                                     float* __restrict__ state_out, int group_stride,
                                                     int table_floats) {
  extern __shared__ float smem[];
  rollout_item<G>(*inst, 0, group_stride, table_floats, smem, steps, state_out);
}

// The state predictions of a batch of ticks (instances whose trees take G
// lanes), one workgroup per item; the LDS layout is sized for the largest.
template <int G>
__global__ __launch_bounds__(64) void predict_batch_kernel(const PredItem* __restrict__ items, int group_stride,
                                                           int table_floats) {
  extern __shared__ float smem[];
  const PredItem it = items[blockIdx.x];
  rollout_item<G>(*it.inst, 0, group_stride, table_floats, smem, it.steps, it.state_out);
}

// Persistent form: a grid sized to the resident wavefronts; each wavefront takes
// work items from a device counter until the table is exhausted (every wavefront
// reaches that exit).  Which wavefront runs an item does not change its result.
// The same depth and legged-tree specialisations as rollout_kernel, and the same
// two wavefronts per SIMD: the lane index is made opaque once per item (see
// rollout_item's per_item), so nothing derived from it stays live across items.
template <int G, int D, int LEG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void rollout_persistent_kernel(
    const DevInst* __restrict__ insts, const int2* __restrict__ work, int n_items, unsigned int* __restrict__ counter,
    int group_stride, int table_floats) {
  extern __shared__ float smem[];
  for (;;) {
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    int item = 0;
    if (lane == 0) item = (int)atomicAdd(counter, 1u);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= n_items) break;
    const int2 w = work[item];
    const DevInst& I = insts[w.x];
    rollout_item<G, D, false, LEG>(I, w.y, group_stride, table_floats, smem, I.H, nullptr, nullptr, nullptr, true);
  }
}

// ---------------------------------------------------------------------------
// Team schedule: every chain of the heavy-path decomposition owns a block of B
// lanes (B = 4 or 8, holding the chain's bodies).  The per-body work runs one
// body per lane of its chain's block (PD law, inertia, bias, contacts, running
// cost, integration); the three sweeps run per chain, one body per level, on the
// block's first three lanes together: lane k holds component k of every
// 3-vector and row k of every 3x3 block with its columns in rotated order
// (entry i is column k + i), and the lanes meet through DPP permutations inside
// their quad.  A cyclic relabelling of the axes is a proper rotation, so a cross
// product keeps its form in every lane: (a x b)_k = a_{k+1} b_{k+2} - a_{k+2} b_{k+1}.
// Sums over the three lanes are taken in the order 0, 1, 2 in every lane, so the
// lanes of a team agree bit for bit on every shared scalar.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float qperm(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ float qr1(float x) { return qperm<0xC9>(x); }  // component k + 1 (quad_perm 1,2,0,3)
__device__ __forceinline__ float qr2(float x) { return qperm<0xD2>(x); }  // component k + 2 (quad_perm 2,0,1,3)
__device__ __forceinline__ float qsum3(float x) { return (qperm<0x00>(x) + qperm<0x55>(x)) + qperm<0xAA>(x); }

// frame of one body as seen by coordinate lane k: rotated row k of R, p_k, v_k, beta_k
struct TFrame {
  float R[3], p, va, vl, ba, bl;
};

// Forward kinematics of a revolute body (as fk_joint) from the parent's frame P:
// tc = the body's team constants for this lane; outputs the frame O, e_k, ax_k, c_k.
__device__ __forceinline__ void team_fk(const float* tc, float cq, float sq, float qd, const TFrame& P, TFrame& O,
                                        float& e, float& ax, float& ca, float& cl) {
  float C[3], C1[3], C2[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) C[i] = tc[i] + cq * tc[3 + i] + sq * tc[6 + i];
#pragma unroll
  for (int i = 0; i < 3; ++i) { C1[i] = qr1(C[i]); C2[i] = qr2(C[i]); }
  // R = Rl C: entry j = sum_m Rl[k][k+m] C[k+m][k+j]; lane k+m holds C[k+m][.] rotated by its own index
#pragma unroll
  for (int j = 0; j < 3; ++j) O.R[j] = P.R[0] * C[j] + P.R[1] * C1[(j + 2) % 3] + P.R[2] * C2[(j + 1) % 3];
  e = P.R[0] * tc[9] + P.R[1] * tc[10] + P.R[2] * tc[11];
  ax = P.R[0] * tc[12] + P.R[1] * tc[13] + P.R[2] * tc[14];
  O.p = P.p + e;
  const float e1 = qr1(e), e2 = qr2(e);
  const float w1 = qr1(P.va), w2 = qr2(P.va);
  O.va = P.va + ax * qd;
  O.vl = P.vl + (w1 * e2 - w2 * e1);
  const float aq = ax * qd, aq1 = qr1(aq), aq2 = qr2(aq);
  const float va1 = qr1(O.va), va2 = qr2(O.va), vl1 = qr1(O.vl), vl2 = qr2(O.vl);
  ca = va1 * aq2 - va2 * aq1;
  cl = vl1 * aq2 - vl2 * aq1;
  const float b1 = qr1(P.ba), b2 = qr2(P.ba);
  O.ba = P.ba + ca;
  O.bl = P.bl + (b1 * e2 - b2 * e1) + cl;
}

// Articulated-body step of a revolute joint (as backward_joint).  Rows of lane k:
// A[i] = A[k][k+i], B[i] = B[k][k+i], T[i] = B[k+i][k], C[i] = C[k][k+i] of the
// articulated inertia [[A, B], [B^T, C]] and the bias (pa, pl); the carried
// inertia and bias come out in the same form.
__device__ __forceinline__ void team_backward(const float* A, const float* B, const float* T, const float* C,
                                              float pa, float pl, float ax, float e, float ca, float cl, float tau,
                                              float arm, float gain, float& Ua, float& Ul, float& invD, float& u,
                                              float* Ap, float* Bp, float* Tp, float* Cp, float& ppa, float& ppl) {
  const float ax1 = qr1(ax), ax2 = qr2(ax);
  Ua = A[0] * ax + A[1] * ax1 + A[2] * ax2;
  Ul = T[0] * ax + T[1] * ax1 + T[2] * ax2;
  const float Dv = (arm + gain) + qsum3(ax * Ua);
  invD = rcp(Dv);
  u = tau - qsum3(ax * pa);
  // Ia = IA - U W^T, W = U / D
  const float Wa = Ua * invD, Wl = Ul * invD;
  const float Wa1 = qr1(Wa), Wa2 = qr2(Wa), Wl1 = qr1(Wl), Wl2 = qr2(Wl), Ua1 = qr1(Ua), Ua2 = qr2(Ua);
  const float IA_[3] = {A[0] - Ua * Wa, A[1] - Ua * Wa1, A[2] - Ua * Wa2};
  const float IB[3] = {B[0] - Ua * Wl, B[1] - Ua * Wl1, B[2] - Ua * Wl2};
  const float IT[3] = {T[0] - Ua * Wl, T[1] - Ua1 * Wl, T[2] - Ua2 * Wl};
  const float IC[3] = {C[0] - Ul * Wl, C[1] - Ul * Wl1, C[2] - Ul * Wl2};
  // pa = pA + Ia c + U u / D
  const float ca1 = qr1(ca), ca2 = qr2(ca), cl1 = qr1(cl), cl2 = qr2(cl);
  const float iqa = IA_[0] * ca + IA_[1] * ca1 + IA_[2] * ca2 + IB[0] * cl + IB[1] * cl1 + IB[2] * cl2;
  const float iql = IT[0] * ca + IT[1] * ca1 + IT[2] * ca2 + IC[0] * cl + IC[1] * cl1 + IC[2] * cl2;
  const float uD = u * invD;
  const float pa2 = pa + iqa + Ua * uD, pl2 = pl + iql + Ul * uD;
  // carried to the parent origin: B' = B + E C, A' = A - B'E - (BE)^T, C' = C (E = e^x)
  const float e1 = qr1(e), e2 = qr2(e);
  float IC1[3], IC2[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) { IC1[i] = qr1(IC[i]); IC2[i] = qr2(IC[i]); }
#pragma unroll
  for (int i = 0; i < 3; ++i) Bp[i] = IB[i] + e1 * IC2[(i + 1) % 3] - e2 * IC1[(i + 2) % 3];
  Tp[0] = Bp[0];
  Tp[1] = qr1(Bp[2]);
  Tp[2] = qr2(Bp[1]);
  const float er[3] = {e, e1, e2};
  float y[3], z[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    y[j] = Bp[(j + 1) % 3] * er[(j + 2) % 3] - Bp[(j + 2) % 3] * er[(j + 1) % 3];
    z[j] = IB[(j + 1) % 3] * er[(j + 2) % 3] - IB[(j + 2) % 3] * er[(j + 1) % 3];
  }
  Ap[0] = IA_[0] - y[0] - z[0];
  Ap[1] = IA_[1] - y[1] - qr1(z[2]);
  Ap[2] = IA_[2] - y[2] - qr2(z[1]);
#pragma unroll
  for (int i = 0; i < 3; ++i) Cp[i] = IC[i];
  const float p1 = qr1(pl2), p2 = qr2(pl2);
  ppa = pa2 + (e1 * p2 - e2 * p1);
  ppl = pl2;
}

// Accelerations of a revolute joint (as forward_joint) from the parent's a' (ala, all).
__device__ __forceinline__ float team_forward(float ala, float all, float e, float ax, float ca, float cl, float Ua,
                                              float Ul, float invD, float u, float& aa, float& al) {
  const float a1 = qr1(ala), a2 = qr2(ala), e1 = qr1(e), e2 = qr2(e);
  aa = ala + ca;
  al = all + (a1 * e2 - a2 * e1) + cl;
  const float qdd = (u - qsum3(Ua * aa + Ul * al)) * invD;
  aa = aa + ax * qdd;
  return qdd;
}

// Per-lane roles of the team schedule.
struct TeamRole {
  int c, bl, k;            // chain, lane in the chain's block, coordinate lane (0 for lanes past the third)
  int b, slot;             // body of a body lane and its record slot (0 otherwise: never written)
  int cfirst, cpar, pslot; // depth of the chain's first body, its parent (-1: a root) and the parent's slot
  bool body_lane, team;
};

// Body constants a body lane of the team schedule reads.
struct TeamBody {
  float com[3], Ic[6], mass, kp, kd, taumax, q0;
  int c_begin, c_count;
};
__device__ __forceinline__ void load_team_body(const DevModel& M, const DevInst* I, const TeamRole& r, TeamBody& c) {
  const int bb = r.b;
  const int j = bb - M.fb;
  const bool joint = r.body_lane && j >= 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) c.com[k] = M.com[bb][k];
#pragma unroll
  for (int k = 0; k < 6; ++k) c.Ic[k] = M.Ic[bb][k];
  c.mass = M.mass[bb];
  c.kp = joint ? M.kp[j] : 0.f;
  c.kd = joint ? M.kd[j] : 0.f;
  c.taumax = joint ? M.taumax[j] : 0.f;
  c.q0 = (joint && I && I->cost_kind == 1) ? I->q0[j] : 0.f;
  c.c_begin = M.c_begin[bb];
  c.c_count = r.body_lane ? M.c_count[bb] : 0;
}

// Stage the team constants (by slot) and the table of the slot of chain c's body at
// depth d (or -1) after the model table.
__device__ __forceinline__ void stage_team_table(const DevModel& M, float* tab, int lane) {
  float* tt = tab + body_table_floats(M.nc);
  const int n = M.nb * kTeamRow;
  for (int i = lane; i < n; i += 64) {
    const int b = i / kTeamRow, w = i % kTeamRow;
    tt[M.team_slot[b] * kTeamSlot + (w / 16) * kTeamK + (w % 16)] = M.team_rows[b][w];
  }
  int* tcb = reinterpret_cast<int*>(tt + M.team_slots * kTeamSlot);
  for (int i = lane; i < kMaxChains * kMaxLevels; i += 64) {
    const int bb = M.chain_body[i / kMaxLevels][i % kMaxLevels];
    tcb[i] = bb >= 0 ? M.team_slot[bb] : -1;
  }
  wave_sync();
}

__device__ __forceinline__ void get16(const float* s, float* d) {
  const float4 a = get4(s), b = get4(s + 4), c = get4(s + 8), e = get4(s + 12);
  d[0] = a.x; d[1] = a.y; d[2] = a.z; d[3] = a.w; d[4] = b.x; d[5] = b.y; d[6] = b.z; d[7] = b.w;
  d[8] = c.x; d[9] = c.y; d[10] = c.z; d[11] = c.w; d[12] = e.x; d[13] = e.y; d[14] = e.z; d[15] = e.w;
}

// What a coordinate lane reads for one level of the backward sweep (loaded a
// level ahead; zeros where the chain has no body at that depth).
struct TeamBwdIn {
  float ir[16], lr[4], tau, gain, arm;
  uint32_t side;
  bool act;
};
__device__ __forceinline__ int team_load_bwd(const TeamRole& r, const int* tcb, const float* tt, const float* ir,
                                             const float* lr, const float* br, int d, int k, TeamBwdIn& o) {
  const int s = r.team ? tcb[r.c * kMaxLevels + d] : -1;
  o.act = s >= 0;
  if (o.act) {
    get16(ir + s * kTeamSlot + k * kTeamK, o.ir);
    const float4 l4 = get4(lr + s * kFrSlot + k * 8);
    o.lr[0] = l4.x; o.lr[1] = l4.y; o.lr[2] = l4.z; o.lr[3] = l4.w;
    const float4 b4 = get4(br + s * 8);
    o.tau = b4.w;
    o.gain = br[s * 8 + 4];
    o.arm = tt[s * kTeamSlot + 15];
    o.side = (uint32_t)__float_as_int(tt[s * kTeamSlot + kTeamK + 15]);
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) o.ir[q] = 0.f;
    o.lr[0] = o.lr[1] = o.lr[2] = o.lr[3] = 0.f;
    o.tau = o.gain = o.arm = 0.f;
    o.side = 0u;
  }
  return s;
}
// the same for the forward sweep
struct TeamFwdIn {
  float lr[8];
  uint32_t side;
  bool act;
};
__device__ __forceinline__ int team_load_fwd(const TeamRole& r, const int* tcb, const float* tt, const float* lr,
                                             int d, int k, TeamFwdIn& o) {
  const int s = r.team ? tcb[r.c * kMaxLevels + d] : -1;
  o.act = s >= 0;
  if (o.act) {
    const float4 l0 = get4(lr + s * kFrSlot + k * 8), l1 = get4(lr + s * kFrSlot + k * 8 + 4);
    o.lr[0] = l0.x; o.lr[1] = l0.y; o.lr[2] = l0.z; o.lr[3] = l0.w;
    o.lr[4] = l1.x; o.lr[5] = l1.y; o.lr[6] = l1.z; o.lr[7] = l1.w;
    o.side = (uint32_t)__float_as_int(tt[s * kTeamSlot + kTeamK + 15]);
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) o.lr[q] = 0.f;
    o.side = 0u;
  }
  return s;
}

// One physics step of the team schedule (same stages and formulas as physics_step):
// tt = team constants and tcb = chain-body table in LDS.  Every coordinate-lane
// computation runs with all lanes active (the DPP permutations need them); the
// lanes of a level without a body compute on zeros and store nothing.
template <int D>
__device__ __attribute__((always_inline)) void team_step(const StepConst& sc, const TeamBody& tb, const float* tab,
                                                         const float* tt, const int* tcb,
                          float* __restrict__ gs, const TeamLayout& L, const TeamRole& r, StepIO& io, bool want_cost,
                          bool terminal = false) {
  float* br = gs + L.br;
  float* fr = gs + L.fr;
  float* lr = gs + L.lr;
  float* ir = gs + L.ir;
  float* pr = gs + L.pr;
  float* ar = gs + L.ar;
  float* bs = gs + L.bs;
  float* gr = gs + L.gr;
  const int fb = sc.fb, b = r.b, k = r.k, sl = r.slot;
  const bool is_base = r.body_lane && fb && b == 0;
  const bool is_joint = r.body_lane && !is_base;
  const int maxd = D > 0 ? D : sc.max_depth;

  // ---- PD law, joint trigonometry, frame B
  float tau = 0.f, gain = 0.f;
  if (is_joint) pd_law(tb.kp, tb.kd, tb.taumax, io.dt, io.q, io.v, io.qref, io.vref, tau, gain);
  io.tau = tau;
  float base_term = 0.f;
  if (want_cost && is_base && sc.cost_kind == 1) base_term = base_cost_term(sc, io.bq);
  if (is_joint) {
    float cq, sq;
    sincosf(io.q, &sq, &cq);
    put4(br + sl * 8, cq, sq, io.v, tau);
    br[sl * 8 + 4] = gain;
  }
  if (is_base) {
    float R[9];
    quat_R(io.bq + 3, R);
#pragma unroll
    for (int q = 0; q < 9; ++q) bs[q] = R[q];
    bs[9] = io.bq[0]; bs[10] = io.bq[1]; bs[11] = io.bq[2];
#pragma unroll
    for (int q = 0; q < 6; ++q) bs[12 + q] = io.bv[q];
  }
  if (!fb && r.c == 0 && r.bl == 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q) bs[q] = (q % 4 == 0) ? 1.f : 0.f;
#pragma unroll
    for (int q = 9; q < 18; ++q) bs[q] = 0.f;
  }
  wave_sync();

  // ---- forward kinematics, one body of each chain per level, on the chain's coordinate lanes
  TFrame F;  // this chain's previous body (the base for chain 0 of a floating base)
  F.R[0] = 1.f; F.R[1] = 0.f; F.R[2] = 0.f;
  F.p = 0.f; F.ba = 0.f; F.bl = 0.f;
  F.va = fb ? bs[12 + k] : 0.f;
  F.vl = fb ? bs[15 + k] : 0.f;
#pragma unroll kLevelUnroll<D>
  for (int d = 1; d <= maxd; ++d) {
    const int sd = r.team ? tcb[r.c * kMaxLevels + d] : -1;  // slot of this chain's body at depth d
    const bool act = sd >= 0;
    float tc[16];
    float4 s4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (act) {
      get16(tt + sd * kTeamSlot + k * kTeamK, tc);
      s4 = get4(br + sd * 8);
    } else {
#pragma unroll
      for (int q = 0; q < 16; ++q) tc[q] = 0.f;
    }
    TFrame P = F;
    if (act && d == r.cfirst) {  // a chain's first body: its parent is elsewhere
      if (r.cpar < 0) {
        P.R[0] = 1.f; P.R[1] = 0.f; P.R[2] = 0.f;
        P.p = P.va = P.vl = P.ba = P.bl = 0.f;
      } else if (fb && r.cpar == 0) {
        P.R[0] = 1.f; P.R[1] = 0.f; P.R[2] = 0.f;
        P.p = 0.f; P.va = bs[12 + k]; P.vl = bs[15 + k]; P.ba = 0.f; P.bl = 0.f;
      } else {
        const float4 f0 = get4(fr + r.pslot * kFrSlot + k * 8), f1 = get4(fr + r.pslot * kFrSlot + k * 8 + 4);
        P.R[0] = f0.x; P.R[1] = f0.y; P.R[2] = f0.z; P.p = f0.w;
        P.va = f1.x; P.vl = f1.y; P.ba = f1.z; P.bl = f1.w;
      }
    }
    TFrame O;
    float e, ax, ca, cl;
    team_fk(tc, s4.x, s4.y, s4.z, P, O, e, ax, ca, cl);
    if (act) {
      put4(fr + sd * kFrSlot + k * 8, O.R[0], O.R[1], O.R[2], O.p);
      put4(fr + sd * kFrSlot + k * 8 + 4, O.va, O.vl, O.ba, O.bl);
      put4(lr + sd * kFrSlot + k * 8, e, ax, ca, cl);
    }
    F = O;
    wave_sync();
  }

  // ---- every body lane: its frame, rigid inertia, bias force, contacts and running cost
  // (every lane reads its slot's record, so the values are chosen, not the memory)
  float R[9], p[3], v[6], beta[6];
#pragma unroll
  for (int kk = 0; kk < 3; ++kk) {
    const float4 f0 = get4(fr + sl * kFrSlot + kk * 8), f1 = get4(fr + sl * kFrSlot + kk * 8 + 4);
    R[kk * 3 + kk] = is_joint ? f0.x : 1.f;
    R[kk * 3 + (kk + 1) % 3] = is_joint ? f0.y : 0.f;
    R[kk * 3 + (kk + 2) % 3] = is_joint ? f0.z : 0.f;
    p[kk] = is_joint ? f0.w : 0.f;
    v[kk] = is_joint ? f1.x : bs[12 + kk];  // the base: its twist (frame B)
    v[3 + kk] = is_joint ? f1.y : bs[15 + kk];
    beta[kk] = is_joint ? f1.z : 0.f;
    beta[3 + kk] = is_joint ? f1.w : 0.f;
  }
  float Rb[9], pb[3];
#pragma unroll
  for (int q = 0; q < 9; ++q) Rb[q] = bs[q];
  pb[0] = bs[9]; pb[1] = bs[10]; pb[2] = bs[11];
  float lane_cost = 0.f;
  if (terminal) {
    if (r.body_lane && sc.cost_kind == 0 && b == sc.ee_body) {
      const float dz = ee_height_error(R, p, sc.ee_pos, Rb, pb, sc.z_des);
      lane_cost = sc.w_ee * dz * dz;
    }
    io.cost = lane_cost;
    io.mask = 0u;
    wave_sync();
    return;
  }
  const float g = sc.g;
  const float agl[3] = {-g * Rb[6], -g * Rb[7], -g * Rb[8]};
  uint32_t mask = 0u;
  if (r.body_lane) {
    float IA[21], pA[6];
    if (is_base) {
      const float eye[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
      body_inertia(eye, tb.com, tb.Ic, tb.mass, IA);
    } else {
      body_inertia(R, tb.com, tb.Ic, tb.mass, IA);
    }
    bias_force(IA, v, pA);
    const int c0 = tb.c_begin, cn = tb.c_count;
    for (int ci = c0; ci < c0 + cn; ++ci) {
      const float* ct = tab + kTabContacts + ci * kCt;
      float vw[3], fw[3];
      const float fn = contact_point(ct, R, p, v, beta, Rb, pb, agl, io.dt, sc.law, IA, pA, vw, fw);
      if (fn > 0.f) mask |= 1u << __float_as_int(ct[4]);
      if (want_cost && sc.cost_kind == 1) contact_cost(sc, fn, vw, fw, ct[3], lane_cost);
    }
    if (want_cost) body_cost(sc, b, is_base, is_joint, base_term, io.q, tb.q0, tau, R, p, Rb, pb, lane_cost);
    // rows for the coordinate lanes
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      float* d = ir + sl * kTeamSlot + kk * kTeamK;
      const int c1 = (kk + 1) % 3, c2 = (kk + 2) % 3;
      put4(d, IA[SI(kk, kk)], IA[SI(kk, c1)], IA[SI(kk, c2)], IA[SI(kk, 3 + kk)]);
      put4(d + 4, IA[SI(kk, 3 + c1)], IA[SI(kk, 3 + c2)], IA[SI(kk, 3 + kk)], IA[SI(c1, 3 + kk)]);
      put4(d + 8, IA[SI(c2, 3 + kk)], IA[SI(3 + kk, 3 + kk)], IA[SI(3 + kk, 3 + c1)], IA[SI(3 + kk, 3 + c2)]);
      put4(d + 12, pA[kk], pA[3 + kk], 0.f, 0.f);
    }
  }
  io.cost = lane_cost;
  io.mask = mask;
  wave_sync();

  // ---- backward sweep, leaves to root, on the coordinate lanes
  float cA[3] = {0.f, 0.f, 0.f}, cB[3] = {0.f, 0.f, 0.f}, cT[3] = {0.f, 0.f, 0.f}, cC[3] = {0.f, 0.f, 0.f};
  float cpa = 0.f, cpl = 0.f;  // carried by this chain's deeper body

#pragma unroll kLevelUnrollRoot<D>
  for (int d = maxd; d >= 0; --d) {
    TeamBwdIn cur;
    const int sd = team_load_bwd(r, tcb, tt, ir, lr, br, d, k, cur);
    const bool act = cur.act;
    float A[3] = {cur.ir[0], cur.ir[1], cur.ir[2]}, B[3] = {cur.ir[3], cur.ir[4], cur.ir[5]};
    float T[3] = {cur.ir[6], cur.ir[7], cur.ir[8]}, C[3] = {cur.ir[9], cur.ir[10], cur.ir[11]};
    float pa = cur.ir[12], pl = cur.ir[13];
    const float e = cur.lr[0], ax = cur.lr[1], ca = cur.lr[2], cl = cur.lr[3];
    const float tau_d = cur.tau, gain_d = cur.gain, arm_d = cur.arm;
    uint32_t side = cur.side;
    const bool deeper = act && d < maxd && tcb[r.c * kMaxLevels + d + 1] >= 0;  // the chain goes on
    if (deeper) {
#pragma unroll
      for (int i = 0; i < 3; ++i) { A[i] += cA[i]; B[i] += cB[i]; T[i] += cT[i]; C[i] += cC[i]; }
      pa += cpa;
      pl += cpl;
    }
    while (side) {
      const int c2 = __builtin_ctz(side);
      side &= side - 1u;
      float q[16];
      get16(pr + c2 * kTeamSlot + k * kTeamK, q);
      A[0] += q[0]; A[1] += q[1]; A[2] += q[2]; B[0] += q[3];
      B[1] += q[4]; B[2] += q[5]; T[0] += q[6]; T[1] += q[7];
      T[2] += q[8]; C[0] += q[9]; C[1] += q[10]; C[2] += q[11];
      pa += q[12]; pl += q[13];
    }
    float Ua, Ul, invD, u, nA[3], nB[3], nT[3], nC[3], npa, npl;
    team_backward(A, B, T, C, pa, pl, ax, e, ca, cl, tau_d, arm_d, gain_d, Ua, Ul, invD, u, nA, nB, nT, nC, npa,
                  npl);
    const bool base_here = act && fb && d == 0;
    if (act && !base_here) {
      put4(lr + sd * kFrSlot + k * 8 + 4, Ua, Ul, invD, u);
      if (d == r.cfirst && r.cpar >= 0) {
        float* q = pr + r.c * kTeamSlot + k * kTeamK;
        put4(q, nA[0], nA[1], nA[2], nB[0]);
        put4(q + 4, nB[1], nB[2], nT[0], nT[1]);
        put4(q + 8, nT[2], nC[0], nC[1], nC[2]);
        put4(q + 12, npa, npl, 0.f, 0.f);
      }
    }
    if (base_here) {  // the floating base: its rows go to the solve
      float* q = gr + k * kTeamK;
      put4(q, A[0], A[1], A[2], B[0]);
      put4(q + 4, B[1], B[2], T[0], T[1]);
      put4(q + 8, T[2], C[0], C[1], C[2]);
      put4(q + 12, pa, pl, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) { cA[i] = nA[i]; cB[i] = nB[i]; cT[i] = nT[i]; cC[i] = nC[i]; }
    cpa = npa;
    cpl = npl;
    wave_sync();
  }

  // ---- root: floating base solves IA0 a0' = -pA0
  if (is_base) {
    float IA[21], pA[6], a0[6];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      const float* q = gr + kk * kTeamK;
      const int c1 = (kk + 1) % 3, c2 = (kk + 2) % 3;
      IA[SI(kk, kk)] = q[0];
      if (kk <= c1) IA[SI(kk, c1)] = q[1];
      if (kk <= c2) IA[SI(kk, c2)] = q[2];
      IA[SI(kk, 3 + kk)] = q[3]; IA[SI(kk, 3 + c1)] = q[4]; IA[SI(kk, 3 + c2)] = q[5];
      IA[SI(3 + kk, 3 + kk)] = q[9];
      if (kk <= c1) IA[SI(3 + kk, 3 + c1)] = q[10];
      if (kk <= c2) IA[SI(3 + kk, 3 + c2)] = q[11];
      pA[kk] = q[12];
      pA[3 + kk] = q[13];
    }
    base_solve(IA, pA, a0);
#pragma unroll
    for (int q = 0; q < 6; ++q) bs[18 + q] = a0[q];
    io.ba[0] = a0[0]; io.ba[1] = a0[1]; io.ba[2] = a0[2];
    io.ba[3] = a0[3] + agl[0]; io.ba[4] = a0[4] + agl[1]; io.ba[5] = a0[5] + agl[2];
  }
  wave_sync();

  // ---- forward sweep, root to leaves, on the coordinate lanes
  float Fa = fb ? bs[18 + k] : 0.f, Fl = fb ? bs[21 + k] : 0.f;  // chain 0 starts at the base
#pragma unroll kLevelUnroll<D>
  for (int d = 1; d <= maxd; ++d) {
    TeamFwdIn cur;
    const int sd = team_load_fwd(r, tcb, tt, lr, d, k, cur);
    const bool act = cur.act;
    const float* lf = cur.lr;
    const uint32_t side = cur.side;
    float ala = Fa, all = Fl;
    if (act && d == r.cfirst) {
      if (r.cpar < 0) {  // fixed world: a' = -a_g = (0, 0, 0, 0, 0, g)
        ala = 0.f;
        all = k == 2 ? g : 0.f;
      } else if (fb && r.cpar == 0) {
        ala = bs[18 + k];
        all = bs[21 + k];
      } else {
        const float2 a2 = *reinterpret_cast<const float2*>(ar + r.pslot * 8 + k * 2);
        ala = a2.x;
        all = a2.y;
      }
    }
    float aa, al;
    const float qdd = team_forward(ala, all, lf[0], lf[1], lf[2], lf[3], lf[4], lf[5], lf[6], lf[7], aa, al);
    if (act) {
      if (side != 0u) *reinterpret_cast<float2*>(ar + sd * 8 + k * 2) = make_float2(aa, al);
      if (k == 0) br[sd * 8 + 5] = qdd;
    }
    Fa = aa;
    Fl = al;
    wave_sync();
  }
  io.qdd = is_joint ? br[sl * 8 + 5] : 0.f;
}

// Fused rollout of one work item on the team schedule (as rollout_item, per_item
// included).
template <int G, int D = 0>
__device__ __attribute__((always_inline)) void team_item(const DevInst& I, int first, int group_stride,
                                                         int table_floats, float* smem, bool per_item = false) {
  int lane = threadIdx.x;
  if (per_item) asm volatile("" : "+v"(lane));
  const int grp = lane / G, l = lane % G;
  const DevModel& M = *I.model;
  float* tab = smem;
  stage_model_table(M, &I, tab, lane);
  stage_team_table(M, tab, lane);
  const float* tt = tab + body_table_floats(M.nc);
  const int* tcb = reinterpret_cast<const int*>(tt + M.team_slots * kTeamSlot);
  const int n = first + grp;
  const bool valid = n < I.N;
  const TeamLayout L = team_layout(G, M.team_slots, I.E, M.n_chains);
  float* gs = smem + table_floats + grp * group_stride;
  float* knots = gs + L.knots;
  float* red = gs + L.red;

  if (I.generate) {
    sample_group<G>(M, I, valid ? n : 0, l, knots, valid, tab);
  } else {
    const float* src = I.samples + (size_t)(valid ? n : 0) * I.E;
    for (int e = l; e < I.E; e += G) knots[e] = src[e];
  }
  wave_sync();

  const StepConst sc = load_step_const(M, &I, 0.f);
  TeamRole r;
  const int B = M.team_block;
  r.c = l / B;
  r.bl = l % B;
  const bool in_chain = r.c < M.n_chains;
  r.team = in_chain && r.bl < 3;
  r.k = r.bl < 3 ? r.bl : 0;
  r.cfirst = in_chain ? M.chain_first[r.c] : 0;
  r.cpar = in_chain ? M.chain_parent[r.c] : -1;
  r.body_lane = in_chain && r.bl < M.chain_len[r.c];
  r.b = r.body_lane ? M.chain_body[r.c][r.cfirst + r.bl] : 0;
  r.slot = r.body_lane ? M.team_slot[r.b] : 0;
  r.pslot = r.cpar >= 0 ? M.team_slot[r.cpar] : 0;
  const int fb = sc.fb, nq = fb ? 7 + M.nu : M.nu;
  const int b = r.b;
  const bool is_joint = r.body_lane && !(fb && b == 0);
  const bool is_base = r.body_lane && fb && b == 0;
  const int j = b - fb;
  StepIO io;
  io.q = io.v = 0.f;
  if (is_joint) {
    io.q = I.x0[(fb ? 7 : 0) + j];
    io.v = I.x0[nq + (fb ? 6 : 0) + j];
  }
#pragma unroll
  for (int q = 0; q < 7; ++q) io.bq[q] = fb ? I.x0[q] : 0.f;
#pragma unroll
  for (int q = 0; q < 6; ++q) io.bv[q] = fb ? I.x0[nq + q] : 0.f;
#pragma unroll
  for (int q = 0; q < 6; ++q) io.ba[q] = 0.f;
  io.qref = io.vref = 0.f;
  io.dt = sc.dt;

  TeamBody tb;
  load_team_body(M, &I, r, tb);
  uint32_t* const masks = I.masks;
  const int H = I.H, F = sc.F, F_run = H * sc.nsub;
  float acc = 0.f;
  StepClock clk;
  HermiteSeg hs{0.f, 0.f, 0.f, 0.f};
  int hseg = -1;
  for (int f = 0; f < F_run; ++f) {
    const bool control = clk.sub == 0;
    if (clk.seg != hseg) {
      hseg = clk.seg;
      if (is_joint) hs = hermite_segment(knots, sc.K, sc.nu, hseg, j, sc.delta);
    }
    if (is_joint) {
      hermite_eval(hs, (float)clk.rem * sc.inv_F, sc.inv_delta, &io.qref, &io.vref);
      if (sc.spline_mode != 0) io.vref = 0.f;
    }
    team_step<D>(sc, tb, tab, tt, tcb, gs, L, r, io, control);
    if (control) {
      acc += io.cost;
      if (masks) {
        const uint32_t mk = group_or<G>(io.mask, red, l);
        if (l == 0 && valid) masks[(size_t)n * H + clk.h] = mk;
      }
    }
    if (is_joint) {
      io.v = fmaf(io.dt, io.qdd, io.v);
      io.q = fmaf(io.dt, io.v, io.q);
    }
    if (is_base) integrate_base(io.bq, io.bv, io.ba, io.dt);
    clk.advance(sc.K, F, sc.nsub);
  }
  // terminal cost
  if (sc.cost_kind == 1) {
    if (is_base) {
      const float T = (float)H * I.dt;
      float e = 0.f;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float target = (q == 2 && I.targets->terminal_z_abs) ? I.targets->z_terminal : I.x0[q] + I.targets->v_des[q] * T;
        e += fabsf(io.bq[q] - target);
      }
      acc += I.w_H * e;
    }
  } else {
    team_step<D>(sc, tb, tab, tt, tcb, gs, L, r, io, false, true);
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
template <int G, int D>
__global__ __launch_bounds__(64) void team_kernel(const DevInst* __restrict__ insts, const int2* __restrict__ work,
                                                  int group_stride, int table_floats) {
  extern __shared__ float smem[];
  constexpr int R = 64 / G;
  const int2 w = work ? work[blockIdx.x] : make_int2(0, (int)blockIdx.x * R);
  const DevInst& I = insts[w.x];
  team_item<G, D>(I, w.y, group_stride, table_floats, smem);
}

// Persistent form (as rollout_persistent_kernel).
template <int G>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void team_persistent_kernel(
    const DevInst* __restrict__ insts, const int2* __restrict__ work, int n_items, unsigned int* __restrict__ counter,
    int group_stride, int table_floats) {
  extern __shared__ float smem[];
  for (;;) {
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    int item = 0;
    if (lane == 0) item = (int)atomicAdd(counter, 1u);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= n_items) break;
    const int2 w = work[item];
    const DevInst& I = insts[w.x];
    team_item<G>(I, w.y, group_stride, table_floats, smem, true);
  }
}

// ---------------------------------------------------------------------------
// Chain schedule: one lane per kinematic chain (heavy-path decomposition of
// the tree), 64/GC rollouts per wavefront.  Per step a lane walks its chain
// root to leaf (Hermite reference, PD law, kinematics), leaf to root (inertia,
// bias, contacts, running cost, articulated-body pass, root solve) and root to
// leaf again (accelerations, integration).  Lanes meet only where a chain
// hangs off another chain's body, through attach and publish slots in LDS; a
// level loop with one body per lane keeps every parent ahead of its children.
// Each body goes through the same helpers in the same order as in the body
// schedule (children added in child-list order, costs summed per body in body
// order), so the two schedules give identical results.
//
// LDS: the model table (body rows, chain bodies, contact rows) once per
// wavefront, then one region per rollout group:
//   rec[nb][kRec]  per body: [0,9) R [9,12) p [12,18) v [18,24) beta [24,27) e
//                  [27,30) ax 30 tau 31 gain; after the backward pass [0,6) U
//                  6 1/D 7 u [8,14) c; and, kept across steps, 32 q 33 qd
//                  34 running cost of the body
//   base[16]       world rotation (9) and position (3) of frame B
//   knots[E]       this rollout's knots
//   pub[nch][kPub] articulated inertia and bias a chain's first body hands to
//                  its parent on another chain
//   att[natt][kAtt] frame (R p v beta) and a' of a body other chains hang off
//   red[GC]        reduction scratch
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ibits(float x) { return __float_as_int(x); }

// Root-to-leaf pass: PD law (unless terminal) and kinematics of every body of
// this lane's chain; publishes frames other chains hang off.
__device__ __forceinline__ void chain_fk(const StepConst& sc, const float* rows, const int* cbody, float* rec,
                                         float* bas, const float* knots, float* att, bool act, int c, int cfirst,
                                         int catt, int nlev, int seg, int rem, bool terminal, const float* bq,
                                         const float* bv) {
  const int fb = sc.fb;
  const float dt = sc.dt;
  float fR[9], fp[3], fv[6], fbt[6];  // frame of this chain's previous body
  for (int d = 0; d < nlev; ++d) {
    const int b = act ? cbody[c * kMaxLevels + d] : -1;
    if (b >= 0) {
      const float* rw = rows + b * kRow;
      float* r = rec + b * kRec;
      if (fb && b == 0) {
        float Rw[9];
        quat_R(bq + 3, Rw);
#pragma unroll
        for (int k = 0; k < 9; ++k) bas[k] = Rw[k];
        bas[9] = bq[0]; bas[10] = bq[1]; bas[11] = bq[2];
#pragma unroll
        for (int k = 0; k < 9; ++k) fR[k] = (k % 4 == 0) ? 1.f : 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) fp[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) { fv[k] = bv[k]; fbt[k] = 0.f; }
#pragma unroll
        for (int k = 0; k < 9; ++k) r[k] = fR[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) r[9 + k] = 0.f;
#pragma unroll
        for (int k = 0; k < 6; ++k) { r[12 + k] = fv[k]; r[18 + k] = 0.f; }
#pragma unroll
        for (int k = 24; k < 32; ++k) r[k] = 0.f;
      } else {
        const int j = b - fb;
        const float q = r[32], qd = r[33];
        float tau = 0.f, gain = 0.f;
        if (!terminal) {
          float qref, vref;
          hermite(knots, sc.K, sc.nu, sc.inv_F, sc.delta, sc.inv_delta, seg, rem, j, &qref, &vref);
          if (sc.spline_mode != 0) vref = 0.f;
          pd_law(rw[row::kp], rw[row::kd], rw[row::taumax], dt, q, qd, qref, vref, tau, gain);
        }
        float Rl[9], pl[3], vl[6], bl[6];
        if (d == cfirst) {
          if (catt >= 0) {
            const float* a = att + catt * kAtt;
#pragma unroll
            for (int k = 0; k < 9; ++k) Rl[k] = a[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) pl[k] = a[9 + k];
#pragma unroll
            for (int k = 0; k < 6; ++k) { vl[k] = a[12 + k]; bl[k] = a[18 + k]; }
          } else {
#pragma unroll
            for (int k = 0; k < 9; ++k) Rl[k] = (k % 4 == 0) ? 1.f : 0.f;
#pragma unroll
            for (int k = 0; k < 3; ++k) pl[k] = 0.f;
#pragma unroll
            for (int k = 0; k < 6; ++k) { vl[k] = 0.f; bl[k] = 0.f; }
          }
        } else {
#pragma unroll
          for (int k = 0; k < 9; ++k) Rl[k] = fR[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) pl[k] = fp[k];
#pragma unroll
          for (int k = 0; k < 6; ++k) { vl[k] = fv[k]; bl[k] = fbt[k]; }
        }
        float cq, sq, C[9];
        sincosf(q, &sq, &cq);
        joint_rotation(rw + row::P, cq, sq, C);
        float e[3], ax[3], cv[6];
        fk_joint(Rl, pl, vl, bl, C, rw + row::p_tree, rw + row::axis_p, qd, fR, fp, e, ax, fv, cv, fbt);
#pragma unroll
        for (int k = 0; k < 9; ++k) r[k] = fR[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) { r[9 + k] = fp[k]; r[24 + k] = e[k]; r[27 + k] = ax[k]; }
#pragma unroll
        for (int k = 0; k < 6; ++k) { r[12 + k] = fv[k]; r[18 + k] = fbt[k]; }
        r[30] = tau;
        r[31] = gain;
      }
      const int aid = ibits(rw[row::att]);
      if (aid >= 0) {
        float* a = att + aid * kAtt;
#pragma unroll
        for (int k = 0; k < 9; ++k) a[k] = fR[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) a[9 + k] = fp[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) { a[12 + k] = fv[k]; a[18 + k] = fbt[k]; }
      }
    }
    wave_sync();
  }
}

// Leaf-to-root pass: inertia, bias, contacts and running cost of each body,
// then the articulated-body step; the floating base solves for its
// acceleration.  Returns this lane's contact activity bits.
__device__ __forceinline__ uint32_t chain_backward(const StepConst& sc, const float* tab, const float* rows,
                                                   const int* cbody, float* rec, const float* bas, float* pub,
                                                   float* att, bool act, int c, int cfirst, int catt, int nlev,
                                                   bool want_cost, float base_term, float* ba, float* ca) {
  const int fb = sc.fb;
  const float dt = sc.dt;
  const float g = sc.g;
  uint32_t mask = 0u;
  float cI[21], cp[6];  // articulated inertia and bias of this chain's deeper body, at this body's origin
  float Rb[9], pb[3];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rb[k] = bas[k];
  pb[0] = bas[9]; pb[1] = bas[10]; pb[2] = bas[11];
  const float agl[3] = {-g * Rb[6], -g * Rb[7], -g * Rb[8]};
  for (int d = nlev - 1; d >= 0; --d) {
    const int b = act ? cbody[c * kMaxLevels + d] : -1;
    if (b >= 0) {
      const float* rw = rows + b * kRow;
      float* r = rec + b * kRec;
      const bool is_base = fb && b == 0;
      float R[9], p[3], v[6], beta[6];
#pragma unroll
      for (int k = 0; k < 9; ++k) R[k] = r[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) p[k] = r[9 + k];
#pragma unroll
      for (int k = 0; k < 6; ++k) { v[k] = r[12 + k]; beta[k] = r[18 + k]; }
      const float tau = r[30], gain = r[31];
      float IA[21], pA[6];
      if (is_base) {
        const float eye[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
        body_inertia(eye, rw + row::com, rw + row::Ic, rw[row::mass], IA);
      } else {
        body_inertia(R, rw + row::com, rw + row::Ic, rw[row::mass], IA);
      }
      bias_force(IA, v, pA);
      float lane_cost = 0.f;
      const int c0 = ibits(rw[row::c_begin]), cn = ibits(rw[row::c_count]);
      for (int ci = c0; ci < c0 + cn; ++ci) {
        const float* ct = tab + kTabContacts + ci * kCt;
        float vw[3], fw[3];
        const float fn = contact_point(ct, R, p, v, beta, Rb, pb, agl, dt, sc.law, IA, pA, vw, fw);
        if (fn > 0.f) mask |= 1u << ibits(ct[4]);
        if (want_cost && sc.cost_kind == 1) contact_cost(sc, fn, vw, fw, ct[3], lane_cost);
      }
      if (want_cost) {
        body_cost(sc, b, is_base, !is_base, base_term, is_base ? 0.f : r[32], rw[row::q0], tau, R, p, Rb, pb,
                  lane_cost);
        r[34] += lane_cost;
      }
      // children in child-list order: the chain's own child from registers, others from their publish slots
      const int nch = ibits(rw[row::n_child]), heavy = ibits(rw[row::heavy]);
      for (int k = 0; k < nch; ++k) {
        const int ch = ibits(rw[row::child + k]);
        if (ch == heavy) {
#pragma unroll
          for (int q = 0; q < 21; ++q) IA[q] += cI[q];
#pragma unroll
          for (int q = 0; q < 6; ++q) pA[q] += cp[q];
        } else {
          const float* s = pub + ibits(rows[ch * kRow + row::chain]) * kPub;
#pragma unroll
          for (int q = 0; q < 21; ++q) IA[q] += s[q];
#pragma unroll
          for (int q = 0; q < 6; ++q) pA[q] += s[21 + q];
        }
      }
      if (!is_base) {
        float e[3], ax[3], cv[6];
#pragma unroll
        for (int k = 0; k < 3; ++k) { e[k] = r[24 + k]; ax[k] = r[27 + k]; }
        vel_product(v, ax, r[33], cv);
        float U[6], invD, u, Ip[21], pp[6];
        backward_joint(IA, pA, ax, cv, e, tau, rw[row::arm], gain, U, invD, u, Ip, pp);
#pragma unroll
        for (int k = 0; k < 6; ++k) { r[k] = U[k]; r[8 + k] = cv[k]; }
        r[6] = invD;
        r[7] = u;
        if (d == cfirst && catt >= 0) {
          float* s = pub + c * kPub;
#pragma unroll
          for (int q = 0; q < 21; ++q) s[q] = Ip[q];
#pragma unroll
          for (int q = 0; q < 6; ++q) s[21 + q] = pp[q];
        } else {
#pragma unroll
          for (int q = 0; q < 21; ++q) cI[q] = Ip[q];
#pragma unroll
          for (int q = 0; q < 6; ++q) cp[q] = pp[q];
        }
      } else {
        float a0[6];
        base_solve(IA, pA, a0);
        ba[0] = a0[0]; ba[1] = a0[1]; ba[2] = a0[2];
        ba[3] = a0[3] + agl[0]; ba[4] = a0[4] + agl[1]; ba[5] = a0[5] + agl[2];
#pragma unroll
        for (int q = 0; q < 6; ++q) ca[q] = a0[q];
        const int aid = ibits(rw[row::att]);
        if (aid >= 0) {
#pragma unroll
          for (int q = 0; q < 6; ++q) att[aid * kAtt + 24 + q] = a0[q];
        }
      }
    }
    wave_sync();
  }
  return mask;
}

// Root-to-leaf pass: joint accelerations and the semi-implicit Euler update of
// the joints (v += dt qdd, q += dt v).
__device__ __forceinline__ void chain_forward(const StepConst& sc, const float* rows, const int* cbody, float* rec,
                                              float* att, bool act, int c, int cfirst, int catt, int nlev, float* ca) {
  const int fb = sc.fb;
  const float dt = sc.dt;
  for (int d = 0; d < nlev; ++d) {
    const int b = act ? cbody[c * kMaxLevels + d] : -1;
    if (b >= 0 && !(fb && b == 0)) {
      const float* rw = rows + b * kRow;
      float* r = rec + b * kRec;
      float al[6];
      if (d == cfirst) {
        if (catt >= 0) {
#pragma unroll
          for (int q = 0; q < 6; ++q) al[q] = att[catt * kAtt + 24 + q];
        } else {
          // fixed world: a' = -a_g = (0, 0, 0, 0, 0, g)
          al[0] = al[1] = al[2] = 0.f; al[3] = 0.f; al[4] = 0.f; al[5] = sc.g;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 6; ++q) al[q] = ca[q];
      }
      float U[6], cv[6], e[3], ax[3];
#pragma unroll
      for (int k = 0; k < 6; ++k) { U[k] = r[k]; cv[k] = r[8 + k]; }
#pragma unroll
      for (int k = 0; k < 3; ++k) { e[k] = r[24 + k]; ax[k] = r[27 + k]; }
      const float qdd = forward_joint(al, e, cv, U, r[7], r[6], ax, ca);
      const int aid = ibits(rw[row::att]);
      if (aid >= 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) att[aid * kAtt + 24 + q] = ca[q];
      }
      const float qd = fmaf(dt, qdd, r[33]);
      r[33] = qd;
      r[32] = fmaf(dt, qd, r[32]);
    }
    wave_sync();
  }
}

template <int GC>
__device__ __attribute__((always_inline)) void chain_item(const DevInst& I, int first, int group_stride,
                                                          int table_floats, int groups, float* smem) {
  const int lane = threadIdx.x;
  const int grp = lane / GC, l = lane % GC;
  const DevModel& M = *I.model;
  const int nb = M.nb, nc = M.nc, fb = M.fb, nch = M.n_chains;

  // model table of this instance (posture and nominal contact forces patched in)
  float* tab = smem;
  stage_model_table(M, &I, tab, lane);
  float* rows = smem + body_table_floats(nc);
  int* cbody = reinterpret_cast<int*>(rows + nb * kRow);
  {
    const float4* src = reinterpret_cast<const float4*>(&M.rows[0][0]);
    float4* dst = reinterpret_cast<float4*>(rows);
    for (int i = lane; i < nb * kRow / 4; i += 64) dst[i] = src[i];
    const int* cb = &M.chain_body[0][0];
    for (int i = lane; i < kMaxChains * kMaxLevels; i += 64) cbody[i] = cb[i];
  }
  wave_sync();
  if (I.cost_kind == 1)
    for (int b = fb + lane; b < nb; b += 64) rows[b * kRow + row::q0] = I.q0[b - fb];
  wave_sync();
  if (grp >= groups) return;  // the LDS budget holds fewer rollout groups than the wavefront has

  const int n = first + grp;
  const bool valid = n < I.N;
  float* gs = smem + table_floats + grp * group_stride;
  float* rec = gs;
  float* bas = rec + nb * kRec;
  float* knots = bas + 16;
  float* pub = knots + ((I.E + 3) & ~3);
  float* att = pub + nch * kPub;
  float* red = att + M.n_att * kAtt;

  if (I.generate) {
    sample_group<GC>(M, I, valid ? n : 0, l, knots, valid, tab);
  } else {
    const float* src = I.samples + (size_t)(valid ? n : 0) * I.E;
    for (int e = l; e < I.E; e += GC) knots[e] = src[e];
  }

  const bool act = l < nch;
  const int c = act ? l : 0;
  const int cfirst = M.chain_first[c], catt = M.chain_att[c];
  const int nlev = M.n_levels;
  const int nq = fb ? 7 + M.nu : M.nu;
  const bool base_lane = act && fb && c == 0;
  for (int d = 0; d < nlev; ++d) {
    const int b = act ? cbody[c * kMaxLevels + d] : -1;
    if (b >= 0) {
      float* r = rec + b * kRec;
      if (!(fb && b == 0)) {
        const int j = b - fb;
        r[32] = I.x0[(fb ? 7 : 0) + j];
        r[33] = I.x0[nq + (fb ? 6 : 0) + j];
      }
      r[34] = 0.f;
    }
  }
  if (!fb && l == 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) bas[k] = (k < 9 && k % 4 == 0) ? 1.f : 0.f;
  }
  float bq[7], bv[6], ba[6], ca[6];
#pragma unroll
  for (int k = 0; k < 7; ++k) bq[k] = fb ? I.x0[k] : 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) { bv[k] = fb ? I.x0[nq + k] : 0.f; ba[k] = 0.f; ca[k] = 0.f; }
  wave_sync();

  const StepConst sc = load_step_const(M, &I, 0.f);
  uint32_t* const masks = I.masks;
  const int H = I.H, F = sc.F;
  StepClock clk;
  for (int f = 0; f < F; ++f) {
    const bool control = clk.sub == 0;
    float base_term = 0.f;
    if (control && base_lane && sc.cost_kind == 1) base_term = base_cost_term(sc, bq);
    chain_fk(sc, rows, cbody, rec, bas, knots, att, act, c, cfirst, catt, nlev, clk.seg, clk.rem, false, bq, bv);
    const uint32_t mask = chain_backward(sc, tab, rows, cbody, rec, bas, pub, att, act, c, cfirst, catt, nlev, control,
                                         base_term, ba, ca);
    chain_forward(sc, rows, cbody, rec, att, act, c, cfirst, catt, nlev, ca);
    if (control && masks) {
      const uint32_t mk = group_or<GC>(mask, red, l);
      if (l == 0 && valid) masks[(size_t)n * H + clk.h] = mk;
    }
    if (base_lane) integrate_base(bq, bv, ba, sc.dt);
    clk.advance(sc.K, F, sc.nsub);
  }

  // terminal cost
  if (sc.cost_kind == 1) {
    if (base_lane) {
      const float T = (float)H * I.dt;
      float e = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float target = (k == 2 && I.targets->terminal_z_abs) ? I.targets->z_terminal : I.x0[k] + I.targets->v_des[k] * T;
        e += fabsf(bq[k] - target);
      }
      rec[34] += I.w_H * e;
    }
  } else {
    // end-effector height at x_H
    chain_fk(sc, rows, cbody, rec, bas, knots, att, act, c, cfirst, catt, nlev, 0, 0, true, bq, bv);
    const int ee = sc.ee_body;
    if (act && ee >= 0 && ibits(rows[ee * kRow + row::chain]) == c) {
      float* r = rec + ee * kRec;
      const float dz = ee_height_error(r, r + 9, sc.ee_pos, bas, bas + 9, sc.z_des);
      const float tc = sc.w_ee * dz * dz;
      r[34] += tc;
    }
  }
  wave_sync();
  if (l == 0 && valid) {
    float S = 0.f;
    for (int b = 0; b < nb; ++b) S += rec[b * kRec + 34];
    if (!isfinite(S)) S = INFINITY;
    I.costs[n] = S;
  }
  wave_sync();
}

// Block = one wavefront holding `groups` (<= 64/GC) rollout groups; work[blockIdx]
// = (instance, first sample) or, when work is null, instance 0 and sample
// blockIdx * groups.
template <int GC>
__global__ __launch_bounds__(64) void chain_kernel(const DevInst* __restrict__ insts, const int2* __restrict__ work,
                                                   int group_stride, int table_floats, int groups) {
  extern __shared__ float smem[];
  const int2 w = work ? work[blockIdx.x] : make_int2(0, (int)blockIdx.x * groups);
  chain_item<GC>(insts[w.x], w.y, group_stride, table_floats, groups, smem);
}

template <int GC>
__global__ __launch_bounds__(64) void chain_persistent_kernel(const DevInst* __restrict__ insts,
                                                              const int2* __restrict__ work, int n_items,
                                                              unsigned int* __restrict__ counter, int group_stride,
                                                              int table_floats, int groups) {
  extern __shared__ float smem[];
  for (;;) {
    int item = 0;
    if (threadIdx.x == 0) item = (int)atomicAdd(counter, 1u);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= n_items) break;
    const int2 w = work[item];
    chain_item<GC>(insts[w.x], w.y, group_stride, table_floats, groups, smem);
    wave_sync();
  }
}

// A new set of task targets for an instance, ordered on the launch stream.
__global__ void set_targets_kernel(DevTargets* __restrict__ dst, DevTargets v) {
  if (threadIdx.x == 0) *dst = v;
}

__global__ void reset_counters(unsigned int* __restrict__ c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = 0u;
}

// ---------------------------------------------------------------------------
// Weighting, update and best tracking.  Grid (the most parts of the launch's
// instances, instances): the workgroups of an instance each take one slice of
// its samples (U.parts of them, update_parts(N)); the workgroups beyond that
// return at once.
// out (per call): the final nominal, best knots and info of the last iteration.
// ---------------------------------------------------------------------------

// The update's workgroups have T threads (64 or 256, update_shape).

// Block-wide sum in a fixed order (tree over threads), deterministic.
template <int T>
__device__ __forceinline__ float block_sum(float x, float* buf) {
  const int t = threadIdx.x;
  buf[t] = x;
  __syncthreads();
  for (int off = T / 2; off > 0; off >>= 1) {
    if (t < off) buf[t] += buf[t + off];
    __syncthreads();
  }
  const float r = buf[0];
  __syncthreads();
  return r;
}

// Sums over one index range of a row-major [*, E] array, V consecutive floats
// (V = 4 or 1) per element block.  The workgroup covers up to T element blocks
// at a time; G = T / min(T, blocks) thread groups take the rows in turn (group
// g: rows g, g + G, ...), each in index order, and their sums are added in
// group order.
template <int V>
struct VecT;
template <>
struct VecT<4> {
  using T = float4;
  static __device__ __forceinline__ float4 zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ void fma(float w, const float4& a, float4& acc) {
    acc.x = fmaf(w, a.x, acc.x); acc.y = fmaf(w, a.y, acc.y); acc.z = fmaf(w, a.z, acc.z); acc.w = fmaf(w, a.w, acc.w);
  }
  static __device__ __forceinline__ void add(const float4& a, float4& acc) {
    acc.x += a.x; acc.y += a.y; acc.z += a.z; acc.w += a.w;
  }
};
template <>
struct VecT<1> {
  using T = float;
  static __device__ __forceinline__ float zero() { return 0.f; }
  static __device__ __forceinline__ void fma(float w, float a, float& acc) { acc = fmaf(w, a, acc); }
  static __device__ __forceinline__ void add(float a, float& acc) { acc += a; }
};

// sum_{n < cnt} w[n] rows[n][:] (w null: weight 1); the result goes to
// emit(element block, value) on threads t < blocks in the chunk.  The element
// blocks are taken NT at a time; each block's rows are split over G threads
// (rows g, g + G, ...), whose sums are then added in g order.  G depends on the
// number of blocks only (NT / EV, at least 1), not on the chunk, so every element
// is added in the same order whichever chunk holds it.
template <int V, int NT, typename Emit>
__device__ __forceinline__ void rows_weighted_sum(const float* __restrict__ rows, int cnt, int E, const float* w,
                                                  float* s_part, Emit emit) {
  using VT = VecT<V>;
  using T = typename VT::T;
  const int t = threadIdx.x, EV = E / V;
  T* part = reinterpret_cast<T*>(s_part);
  const T* col = reinterpret_cast<const T*>(rows);
  constexpr int kIn = 24;  // loads in flight per thread (rows past cnt are not loaded)
  const int G = NT / min(NT, EV);
  for (int e0 = 0; e0 < EV; e0 += NT) {
    const int ec = min(NT, EV - e0);
    const int el = t % ec, g = t / ec, e = e0 + el;
    T acc = VT::zero();
    if (g < G) {
      for (int n = g; n < cnt; n += kIn * G) {
        T a[kIn];
#pragma unroll
        for (int q = 0; q < kIn; ++q) {
          const int r = n + q * G;
          a[q] = r < cnt ? col[(size_t)r * EV + e] : VT::zero();
        }
#pragma unroll
        for (int q = 0; q < kIn; ++q) {
          const int r = n + q * G;
          if (r < cnt) {
            if (w) VT::fma(w[r], a[q], acc);
            else VT::add(a[q], acc);
          }
        }
      }
    }
    __syncthreads();
    if (g < G) part[g * ec + el] = acc;
    __syncthreads();
    if (t < ec) {
      T sum = VT::zero();
      for (int k = 0; k < G; ++k) VT::add(part[k * ec + t], sum);
      emit(e0 + t, sum);
    }
  }
}

// The same sum as rows_weighted_sum<4> over the samples rows n0 .. n0 + cnt - 1,
// with each sample's knots drawn again from the counter-based stream instead of
// read (the rollout kernel then stores none).  Element block b holds positions
// 2b, 2b + 1 and velocities 2b, 2b + 1 (one counter-based block); there are
// E / 4 of them, as many as rows_weighted_sum<4> has, so the rows of every block
// are split over as many threads (G), every element is accumulated over the same
// rows in the same order and the two forms give the same bits (a block may sit
// in another chunk of T blocks than in the stored form; G is the same for every
// chunk).  Needs K nu even and the cubic Hermite knots (velocities sampled, not
// derived).
template <int T>
__device__ __forceinline__ void regen_weighted_sum(const DevInst& I, const float* nom, uint32_t tick, int n0, int cnt,
                                                   const float* w, float* s_part, float* mine) {
  const DevModel& M = *I.model;
  const int t = threadIdx.x, KU = I.K * I.nu, EV = KU / 2;
  const float* sig = I.sigma + I.iter * I.K;
  float4* part = reinterpret_cast<float4*>(s_part);
  const int G = T / min(T, EV);
  for (int e0 = 0; e0 < EV; e0 += T) {
    const int ec = min(T, EV - e0);
    const int el = t % ec, g = t / ec, b = e0 + el;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (g < G) {
      const ElemConst c0 = elem_const(M, I, sig, 2 * b), c1 = elem_const(M, I, sig, 2 * b + 1);
      const float nq0 = nom[2 * b], nq1 = nom[2 * b + 1], nv0 = nom[KU + 2 * b], nv1 = nom[KU + 2 * b + 1];
      // kRow rows are drawn together (independent chains the scheduler can
      // interleave), then added in row order
      constexpr int kRow = 4;
      for (int r0 = g; r0 < cnt; r0 += kRow * G) {
        float4 th[kRow];
#pragma unroll
        for (int q = 0; q < kRow; ++q) {
          const int n = n0 + min(r0 + q * G, cnt - 1);  // rows past the slice are drawn, not added
          const uint4 x = sample_words(I, n, b, tick);
          perturb_element(c0, I.delta, nq0, nv0, n, x.x, x.y, true, th[q].x, th[q].z);
          perturb_element(c1, I.delta, nq1, nv1, n, x.z, x.w, true, th[q].y, th[q].w);
        }
#pragma unroll
        for (int q = 0; q < kRow; ++q) {
          const int r = r0 + q * G;
          if (r < cnt) {
            const float wr = w[r];
            acc.x = fmaf(wr, th[q].x, acc.x); acc.y = fmaf(wr, th[q].y, acc.y);
            acc.z = fmaf(wr, th[q].z, acc.z); acc.w = fmaf(wr, th[q].w, acc.w);
          }
        }
      }
    }
    __syncthreads();
    if (g < G) part[g * ec + el] = acc;
    __syncthreads();
    if (t < ec) {
      float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int k = 0; k < G; ++k) {
        const float4 a = part[k * ec + t];
        sum.x += a.x; sum.y += a.y; sum.z += a.z; sum.w += a.w;
      }
      const int m = 2 * (e0 + t);
      mine[m] = sum.x; mine[m + 1] = sum.y;
      mine[KU + m] = sum.z; mine[KU + m + 1] = sum.w;
    }
  }
}

// Knots of sample n (drawn again, as above) into dst [E].
template <int T>
__device__ __forceinline__ void regen_sample(const DevInst& I, const float* nom, uint32_t tick, int n, float* dst) {
  const DevModel& M = *I.model;
  const int KU = I.K * I.nu;
  const float* sig = I.sigma + I.iter * I.K;
  for (int b = threadIdx.x; b < KU / 2; b += T) {
    const uint4 x = sample_words(I, n, b, tick);
    float q0, v0, q1, v1;
    perturb_element(elem_const(M, I, sig, 2 * b), I.delta, nom[2 * b], nom[KU + 2 * b], n, x.x, x.y, true, q0, v0);
    perturb_element(elem_const(M, I, sig, 2 * b + 1), I.delta, nom[2 * b + 1], nom[KU + 2 * b + 1], n, x.z, x.w,
                    true, q1, v1);
    dst[2 * b] = q0; dst[2 * b + 1] = q1;
    dst[KU + 2 * b] = v0; dst[KU + 2 * b + 1] = v1;
  }
}

// The update of one instance by one workgroup (its part blockIdx.x); o: the
// call's outputs (null fields: not wanted).
template <int T>
__device__ __forceinline__ void update_body(const DevUpdate& U, const UpdateOut o) {
  const int part = blockIdx.x, parts = U.parts;
  if (part >= parts) return;
  const int t = threadIdx.x, N = U.N, E = U.E;
  // the nominal the iteration's samples perturbed (the call's input on its first
  // iteration when the caller's buffer is read in place)
  const float* nom_in = o.nominal_in ? o.nominal_in : U.nominal_in;
  const uint32_t tick = U.regen ? sample_tick(*U.regen) : 0u;  // read before the last part advances it
  __shared__ float s_v[T];
  __shared__ int s_i[T];
  __shared__ float s_x[T];
  __shared__ __align__(16) float s_part[T * 4];
  __shared__ int s_last;
  __shared__ float s_w[(65536 + kUpdMaxParts - 1) / kUpdMaxParts];  // this part's normalised weights (N <= 65536)

  // this part's slice of the samples
  const int slice = (N + parts - 1) / parts;
  const int n0 = part * slice, cnt = max(0, min(N, n0 + slice) - n0);

  // 1. over all samples (every part the same way, so every part gets the same
  //    values): finite minimum (lowest index), maximum and count.  Each thread
  //    takes samples t, t + T, ... in order; up to kReg of them stay in
  //    registers for the weight sum, and the slice's costs go to s_w.
  constexpr int kIn = 8, kReg = 16;
  const bool in_regs = N <= kReg * T;
  const float* costs = U.costs;
  float Sv[kReg];
  float mn = INFINITY, mx = -INFINITY;
  int arg = 0x7fffffff, nf = 0;
  auto visit = [&](float S, int n) {
    if (n >= n0 && n < n0 + cnt) s_w[n - n0] = S;
    if (isfinite(S)) {
      ++nf;
      if (S < mn) { mn = S; arg = n; }
      mx = fmaxf(mx, S);
    }
  };
  if (in_regs) {
#pragma unroll
    for (int q = 0; q < kReg; ++q) {
      const int n = t + q * T;
      Sv[q] = n < N ? costs[n] : INFINITY;
    }
#pragma unroll
    for (int q = 0; q < kReg; ++q) visit(Sv[q], t + q * T);
  } else {
    for (int m0 = t; m0 < N; m0 += kIn * T) {
      float Sq[kIn];
#pragma unroll
      for (int q = 0; q < kIn; ++q) {
        const int n = m0 + q * T;
        Sq[q] = n < N ? costs[n] : INFINITY;
      }
#pragma unroll
      for (int q = 0; q < kIn; ++q) visit(Sq[q], m0 + q * T);
    }
  }
  s_v[t] = mn; s_i[t] = arg; s_x[t] = mx;
  __syncthreads();
  for (int off = T / 2; off > 0; off >>= 1) {
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
  const int nfin = (int)block_sum<T>((float)nf, s_x);

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
  if (in_regs) {
#pragma unroll
    for (int q = 0; q < kReg; ++q) zs += weight(Sv[q]);
  } else {
    for (int m0 = t; m0 < N; m0 += kIn * T) {
      float Sq[kIn];
#pragma unroll
      for (int q = 0; q < kIn; ++q) {
        const int n = m0 + q * T;
        Sq[q] = n < N ? costs[n] : INFINITY;
      }
#pragma unroll
      for (int q = 0; q < kIn; ++q) zs += weight(Sq[q]);
    }
  }
  const float Z = block_sum<T>(zs, s_x);
  const float invZ = nfin > 0 ? 1.f / Z : 0.f;

  // 3. this part's slice: normalised weights (from the costs in s_w), then its
  //    weighted knot sum
  for (int i = t; i < cnt; i += T) {
    const float w = weight(s_w[i]) * invZ;
    s_w[i] = w;
    if (U.weights) U.weights[n0 + i] = w;
  }
  __syncthreads();
  float* mine = U.partial + (size_t)part * E;
  if (U.regen)
    regen_weighted_sum<T>(*U.regen, nom_in, tick, n0, cnt, s_w, s_part, mine);
  else if ((E & 3) == 0)
    rows_weighted_sum<4, T>(U.samples + (size_t)n0 * E, cnt, E, s_w, s_part,
                         [&](int e, float4 v) { reinterpret_cast<float4*>(mine)[e] = v; });
  else
    rows_weighted_sum<1, T>(U.samples + (size_t)n0 * E, cnt, E, s_w, s_part, [&](int e, float v) { mine[e] = v; });

  // 4. the last part to finish adds the slices in part order
  __threadfence();
  __syncthreads();
  if (t == 0) s_last = atomicAdd(U.done, 1u) == (uint32_t)(parts - 1);
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (t == 0) U.done[0] = 0u;  // ready for the next launch
  float* dst = (U.last_iter && o.knots_out) ? o.knots_out : U.nominal_out;
  // the call's running best starts from its input nominal; the best tracking
  // runs before the nominal output is written, since the two may be the same
  // buffer and a drawn-again best sample reads the input nominal
  float* bs = U.best_state;  // [E] knots, then S_best, best_iter, n_nonfinite, all_nonfinite, best_sample
  if (U.first_iter) {
    for (int e = t; e < E; e += T) bs[e] = nom_in[e];
    if (t == 0) {
      bs[E] = INFINITY;
      reinterpret_cast<int*>(bs)[E + 1] = -1;
      reinterpret_cast<int*>(bs)[E + 2] = 0;
      reinterpret_cast<int*>(bs)[E + 3] = 0;
      reinterpret_cast<int*>(bs)[E + 4] = -1;
    }
  }
  __syncthreads();

  // 5. best-sample tracking across the iterations of this call
  const bool improve = nfin > 0 && U.costs[nstar] < bs[E];
  __syncthreads();
  if (improve) {
    if (U.regen) regen_sample<T>(*U.regen, nom_in, tick, nstar, bs);
    else
      for (int e = t; e < E; e += T) bs[e] = U.samples[(size_t)nstar * E + e];
  }
  __syncthreads();
  if (t == 0) {
    if (improve) {
      bs[E] = U.costs[nstar];
      reinterpret_cast<int*>(bs)[E + 1] = U.iter;
      reinterpret_cast<int*>(bs)[E + 4] = nstar;
    }
    reinterpret_cast<int*>(bs)[E + 2] += N - nfin;
    reinterpret_cast<int*>(bs)[E + 3] += nfin == 0 ? 1 : 0;
  }
  __syncthreads();

  // 6. the nominal: the slices added in part order
  if ((E & 3) == 0)
    rows_weighted_sum<4, T>(U.partial, parts, E, nullptr, s_part, [&](int e, float4 v) {
      const float c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) dst[4 * e + k] = nfin > 0 ? c[k] : nom_in[4 * e + k];
    });
  else
    rows_weighted_sum<1, T>(U.partial, parts, E, nullptr, s_part,
                         [&](int e, float v) { dst[e] = nfin > 0 ? v : nom_in[e]; });
  __syncthreads();
  if (U.last_iter) {
    if (o.best_out)
      for (int e = t; e < E; e += T) o.best_out[e] = bs[e];
    if (t == 0 && o.info_out) {
      float* inf = reinterpret_cast<float*>(o.info_out);
      inf[0] = bs[E];
      reinterpret_cast<int*>(inf)[1] = reinterpret_cast<int*>(bs)[E + 1];
      reinterpret_cast<int*>(inf)[2] = reinterpret_cast<int*>(bs)[E + 2];
      reinterpret_cast<int*>(inf)[3] = reinterpret_cast<int*>(bs)[E + 3];
      reinterpret_cast<int*>(inf)[4] = reinterpret_cast<int*>(bs)[E + 4];
    }
  }
  if (U.last_iter && t == 0 && U.tick) U.tick[0] += 1u;
}

template <int T>
__global__ __launch_bounds__(T) void update_kernel(const DevUpdate* __restrict__ ups,
                                                   const UpdateOut* __restrict__ outs, UpdateOut single) {
  update_body<T>(ups[blockIdx.y], outs ? outs[blockIdx.y] : single);
}

// One instance whose descriptor arrives as a kernel argument (no device copy of
// it), with no per-call outputs besides the nominal and the weights.
__global__ __launch_bounds__(kUpdThreads) void update_single_kernel(DevUpdate U) {
  update_body<kUpdThreads>(U, UpdateOut{nullptr, nullptr, nullptr, nullptr});
}
template __global__ void update_kernel<64>(const DevUpdate*, const UpdateOut*, UpdateOut);
template __global__ void update_kernel<256>(const DevUpdate*, const UpdateOut*, UpdateOut);

// Warm start (Sec. III-E): the knots of a trajectory shifted forward by n_steps
// control steps, i.e. its spline at t_k + n_steps dt clamped to the horizon end
// (the final action repeats).  In fine steps of the horizon (F = H n_sub) the
// knot time is k F / (K - 1), so the segment and remainder come from the
// integer m = k F + n_steps n_sub (K - 1) = seg F + rem.  Position-only spline
// variants then take the slopes of the spline through the shifted positions.
// One workgroup; in and out must not alias.

__device__ __forceinline__ void shift_knots_block(const float* __restrict__ in, float* __restrict__ out, int K,
                                                  int nu, int F, int nsub, int n_steps, float delta, int spline_mode,
                                                  float* dg) {
  for (int i = threadIdx.x; i < K * nu; i += kShiftThreads) {
    const int k = i / nu, jj = i % nu;
    const long long m = (long long)k * F + (long long)n_steps * nsub * (K - 1);
    int seg = (int)(m / F), rem = (int)(m - (long long)seg * F);
    if (seg > K - 2) {
      seg = K - 2;
      rem = F;
    }
    float q, v;
    hermite_eval(hermite_segment(in, K, nu, seg, jj, delta), (float)rem / (float)F, 1.f / delta, &q, &v);
    out[i] = q;
    out[K * nu + i] = v;
  }
  if (spline_mode == 0) return;
  if (threadIdx.x == 0 && spline_mode == 1) natural_cubic_diagonal(K, dg);
  __syncthreads();
  for (int jj = threadIdx.x; jj < nu; jj += kShiftThreads) position_spline_slopes(spline_mode, K, nu, jj, delta, dg, out);
}
__global__ __launch_bounds__(kShiftThreads) void shift_knots_kernel(const float* __restrict__ in,
                                                                    float* __restrict__ out, int K, int nu, int F,
                                                                    int nsub, int n_steps, float delta,
                                                                    int spline_mode) {
  __shared__ float dg[kMaxKnots];
  shift_knots_block(in, out, K, nu, F, nsub, n_steps, delta, spline_mode, dg);
}
// The warm-start shifts of a batch of ticks, one workgroup per item.
__global__ __launch_bounds__(kShiftThreads) void shift_batch_kernel(const ShiftItem* __restrict__ items) {
  __shared__ float dg[kMaxKnots];
  const ShiftItem it = items[blockIdx.x];
  shift_knots_block(it.in, it.out, it.K, it.nu, it.F, it.nsub, it.n_steps, it.delta, it.spline_mode, dg);
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

// Two device copies in one launch (block 0: src0 -> dst0, block 1: src1 -> dst1).
__global__ void copy2_kernel(const float* __restrict__ src0, float* __restrict__ dst0, int n0,
                             const float* __restrict__ src1, float* __restrict__ dst1, int n1) {
  const float* src = blockIdx.x == 0 ? src0 : src1;
  float* dst = blockIdx.x == 0 ? dst0 : dst1;
  const int n = blockIdx.x == 0 ? n0 : n1;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
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
  float* tab = smem;  // spline diagonal only
  if (I.spline_mode == 1 && lane == 0) natural_cubic_diagonal(I.K, tab + kTabSpline);
  wave_sync();
  const int n = blockIdx.x * R + grp;
  float* knots = smem + kTabContacts + grp * group_stride + G * kSlot + 16;
  sample_group<G>(*I.model, I, n < I.N ? n : 0, l, knots, n < I.N, tab);
}

template <int G>
__global__ __launch_bounds__(64) void dynamics_kernel(const DevModel* __restrict__ model, int n_states,
                                                      const float* __restrict__ q, const float* __restrict__ v,
                                                      const float* __restrict__ qref, const float* __restrict__ vref,
                                                      float dt, float* __restrict__ qdd, int group_stride,
                                                      int table_floats) {
  extern __shared__ float smem[];
  constexpr int R = 64 / G;
  const int lane = threadIdx.x, grp = lane / G, l = lane % G;
  const DevModel& M = *model;
  float* tab = smem;
  stage_model_table(M, nullptr, tab, lane, true);
  const int s_raw = blockIdx.x * R + grp;
  const bool valid = s_raw < n_states;
  const int s = valid ? s_raw : 0;
  const StepConst sc = load_step_const(M, nullptr, dt);
  const int fb = sc.fb, nu = M.nu, nq = fb ? 7 + nu : nu, nv = fb ? 6 + nu : nu;
  float* gs = smem + table_floats + grp * group_stride;
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
  load_body(M, nullptr, l, body_lane, tab, bc);
  BodyKin kin;  // (unused: the general kernel takes its kinematics fresh)
  physics_step<G>(sc, bc, tab, gs, l, body_lane, io, kin, false);
  if (!valid) return;
  if (is_joint) qdd[(size_t)s * nv + (fb ? 6 : 0) + j] = io.qdd;
  if (fb && l == 0)
    for (int k = 0; k < 6; ++k) qdd[(size_t)s * nv + k] = io.ba[k];
}

// explicit instantiations
#define MPPI_INST(G)                                                                                   \
  template __global__ void rollout_kernel<G, 0, 0>(const DevInst*, const int2*, int, int, const float*,  \
                                                       const float*);                                     \
  template __global__ void rollout_kernel<G, 3, 0>(const DevInst*, const int2*, int, int, const float*,  \
                                                       const float*);                                     \
  template __global__ void rollout_kernel<G, 6, 0>(const DevInst*, const int2*, int, int, const float*,  \
                                                       const float*);                                     \
  template __global__ void rollout_trace_kernel<G, 0, 0>(const DevInst*, const int2*, int, int);     \
  template __global__ void rollout_trace_kernel<G, 3, 0>(const DevInst*, const int2*, int, int);     \
  template __global__ void rollout_trace_kernel<G, 6, 0>(const DevInst*, const int2*, int, int);     \
  template __global__ void rollout_persistent_kernel<G, 0, 0>(const DevInst*, const int2*, int, unsigned int*, int,  \
                                                             int);                                                \
  template __global__ void rollout_persistent_kernel<G, 3, 0>(const DevInst*, const int2*, int, unsigned int*, int,  \
                                                             int);                                                \
  template __global__ void rollout_persistent_kernel<G, 6, 0>(const DevInst*, const int2*, int, unsigned int*, int,  \
                                                             int);                                                \
  template __global__ void sample_kernel<G>(const DevInst*, int);                                      \
  template __global__ void predict_kernel<G>(const DevInst*, int, float*, int, int);                   \
  template __global__ void predict_batch_kernel<G>(const PredItem*, int, int);                         \
  template __global__ void dynamics_kernel<G>(const DevModel*, int, const float*, const float*,        \
                                              const float*, const float*, float, float*, int, int);  \
  template __global__ void team_kernel<G, 0>(const DevInst*, const int2*, int, int);                   \
  template __global__ void team_kernel<G, 3>(const DevInst*, const int2*, int, int);                   \
  template __global__ void team_kernel<G, 6>(const DevInst*, const int2*, int, int);                   \
  template __global__ void team_persistent_kernel<G>(const DevInst*, const int2*, int, unsigned int*, int, int);
// legged trees up to 3 levels deep (a base and 2..10 chains of up to three bodies)
#define MPPI_LEG_INST(G)                                                                               \
  template __global__ void rollout_kernel<G, 3, 1>(const DevInst*, const int2*, int, int, const float*,   \
                                                      const float*);                                      \
  template __global__ void rollout_trace_kernel<G, 3, 1>(const DevInst*, const int2*, int, int);                \
  template __global__ void rollout_persistent_kernel<G, 3, 1>(const DevInst*, const int2*, int, unsigned int*, int,  \
                                                             int);
MPPI_LEG_INST(8)
MPPI_LEG_INST(16)
MPPI_LEG_INST(32)
#undef MPPI_LEG_INST
// fixed-base serial chains up to 3 bodies
#define MPPI_SERIAL_INST(G)                                                                            \
  template __global__ void rollout_kernel<G, 3, 3>(const DevInst*, const int2*, int, int, const float*,   \
                                                      const float*);                                      \
  template __global__ void rollout_trace_kernel<G, 3, 3>(const DevInst*, const int2*, int, int);                \
  template __global__ void rollout_persistent_kernel<G, 3, 3>(const DevInst*, const int2*, int, unsigned int*, int,  \
                                                             int);
MPPI_SERIAL_INST(4)
MPPI_SERIAL_INST(8)
#undef MPPI_SERIAL_INST
// four chains of three bodies on 16 lanes (the quadruped's shape)
template __global__ void rollout_kernel<16, 3, 2>(const DevInst*, const int2*, int, int, const float*, const float*);
template __global__ void rollout_trace_kernel<16, 3, 2>(const DevInst*, const int2*, int, int);
template __global__ void rollout_persistent_kernel<16, 3, 2>(const DevInst*, const int2*, int, unsigned int*, int, int);
MPPI_INST(4)
MPPI_INST(8)
MPPI_INST(16)
MPPI_INST(32)
MPPI_INST(64)
#undef MPPI_INST
#define MPPI_CHAIN_INST(GC)                                                                          \
  template __global__ void chain_kernel<GC>(const DevInst*, const int2*, int, int, int);             \
  template __global__ void chain_persistent_kernel<GC>(const DevInst*, const int2*, int, unsigned int*, int, int, int);
MPPI_CHAIN_INST(1)
MPPI_CHAIN_INST(2)
MPPI_CHAIN_INST(4)
MPPI_CHAIN_INST(8)
#undef MPPI_CHAIN_INST

}  // namespace mppi
