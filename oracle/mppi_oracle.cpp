// mppi_oracle.cpp -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
//
// A plain, slow, scalar CPU reference of the reference-free MPPI step of
// Schramm et al., "Reference-Free Sampling-Based Model Predictive Control"
// (arXiv 2511.19204).  It is used only by tests/, by __graft_entry__.smoke()
// and by the cpu_baseline leg of bench.py, to check the HIP library.  It shares
// no source with the HIP path.  Every routine is templated on the scalar type;
// the checked instantiation is double, and a float instantiation exists only to
// diagnose FP32-vs-FP64 divergence.
//
// Conventions (stated once, used everywhere below):
//  * spatial vectors are (angular; linear), Featherstone's Plucker coordinates;
//  * a floating-base model has body 0 = free base, q = [p(3), quat w,x,y,z (4),
//    joints], v = [omega_body(3), v_body(3), joints] (base twist in base
//    coordinates); a fixed-base model has q = joints, v = joints;
//  * every non-base body carries one revolute joint about a unit axis given in
//    its joint frame; the joint frame sits at p_tree, rotated by R_tree, in the
//    parent body frame; body frame = joint frame rotated by q about the axis;
//  * knots are stored [2][N_k][n_u]: the position block then the velocity block.
//
// Parity unpinned: nothing here is compared against the paper's own robots or
// simulator (not available); each piece is pinned by the closed forms,
// invariants and brute-force checks in tests/test_oracle_*.py.

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>

#include "opcount.hpp"
#endif

extern "C" {

typedef struct {
  int32_t n_bodies;
  int32_t floating_base;
  const int32_t* parent;       // [nb], parent[i] < i, -1 = world
  const double* axis;          // [nb][3] unit joint axis (joint frame)
  const double* R_tree;        // [nb][9] row-major, joint frame in parent frame
  const double* p_tree;        // [nb][3] joint frame origin in parent frame
  const double* mass;          // [nb]
  const double* com;           // [nb][3] centre of mass, body frame
  const double* inertia;       // [nb][6] xx yy zz xy xz yz about the com, body frame
  const double* q_min;         // [n_u]
  const double* q_max;         // [n_u]
  const double* tau_max;       // [n_u]
  const double* kp;            // [n_u]
  const double* kd;            // [n_u]
  int32_t n_contacts;
  const int32_t* contact_body; // [nc]
  const double* contact_pos;   // [nc][3] body frame
  double k_contact, d_contact, mu, eps_fric, gravity;
  int32_t ee_body;
  double ee_pos[3];
  int32_t n_substeps;          // physics steps per control step (>= 1)
  const double* armature;      // [n_u] reflected rotor inertia of each joint, or null (zero)
} orc_model;

typedef struct {
  int32_t n_samples, horizon, n_knots, n_iters;
  double dt, lambda;
  int32_t weight_mode;  // 0 = min-max normalised costs, 1 = raw costs
  int32_t noise_mode;   // 0 = exponential annealing kernel, 1 = linear over knots
  double scale_q, beta1, beta2, sigma_lo, sigma_hi;
  int32_t cost_kind;    // 0 = end-effector height (fixed base), 1 = locomotion
  double w_h, w_or, w_q, w_cv, w_cf, w_eff, w_H, w_ee, w_tau;
  double z_des, v_des[3];
  const double* f0z;      // [nc] reference normal force of each contact point
  const double* q0_cost;  // [n_u]
  int32_t spline_mode;    // 0 = cubic Hermite, 1 = natural cubic, 2 = quadratic (position-only, v_ref = 0)
  double q_des[4];        // base orientation target R_des (w, x, y, z); all zero = identity
  int32_t terminal_z_abs; // 1: the terminal target height is z_terminal instead of p_z(x0) + v_des,z H dt
  double z_terminal;
} orc_params;

}  // extern "C"

namespace orc {

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11): ten rounds of the 4x32 S-box
// with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments
// 0x9E3779B9 / 0xBB67AE85.
// ---------------------------------------------------------------------------
static void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Open-interval uniform from the top 23 bits: ((x >> 9) + 1/2) * 2^-23.
static double uniform01(uint32_t x) { return ((double)(x >> 9) + 0.5) * 0x1p-23; }

// Standard normal pair (position, velocity) for knot slot m of sample n at
// iteration iota of tick `tick`.  Counter = (m / 2, n, iota, tick); the even
// slot uses words 0,1 of the block, the odd slot words 2,3; Box-Muller.
template <class T>
static void knot_normals(uint64_t seed, uint32_t tick, int iota, int n, int m, T* zq, T* zv) {
  uint32_t ctr[4] = {(uint32_t)(m / 2), (uint32_t)n, (uint32_t)iota, tick};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t x[4];
  philox4x32_10(ctr, key, x);
  int w = (m % 2) * 2;
  double ua = uniform01(x[w]), ub = uniform01(x[w + 1]);
  double r = std::sqrt(-2.0 * std::log(ua));
  double ang = 2.0 * M_PI * ub;
  *zq = (T)(r * std::cos(ang));
  *zv = (T)(r * std::sin(ang));
}

// ---------------------------------------------------------------------------
// Small dense linear algebra, plain loops.
// ---------------------------------------------------------------------------
template <class T> using V3 = std::array<T, 3>;
template <class T> using M3 = std::array<T, 9>;   // row-major
template <class T> using V6 = std::array<T, 6>;
template <class T> using M6 = std::array<T, 36>;  // row-major

template <class T> static M3<T> m3_eye() { return M3<T>{1, 0, 0, 0, 1, 0, 0, 0, 1}; }
template <class T> static M3<T> m3_mul(const M3<T>& A, const M3<T>& B) {
  M3<T> C{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = 0;
      for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
      C[i * 3 + j] = s;
    }
  return C;
}
template <class T> static M3<T> m3_T(const M3<T>& A) {
  M3<T> C{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[j * 3 + i];
  return C;
}
template <class T> static V3<T> m3_v(const M3<T>& A, const V3<T>& x) {
  V3<T> y{};
  for (int i = 0; i < 3; ++i) y[i] = A[i * 3 + 0] * x[0] + A[i * 3 + 1] * x[1] + A[i * 3 + 2] * x[2];
  return y;
}
template <class T> static V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return V3<T>{a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
template <class T> static M3<T> skew(const V3<T>& a) {
  return M3<T>{0, -a[2], a[1], a[2], 0, -a[0], -a[1], a[0], 0};
}
// Rotation by angle q about unit axis a (Rodrigues).
template <class T> static M3<T> rot_axis(const V3<T>& a, T q) {
  M3<T> K = skew(a), K2 = m3_mul(K, K), R = m3_eye<T>();
  T s = std::sin(q), c = std::cos(q);
  for (int i = 0; i < 9; ++i) R[i] += s * K[i] + (1 - c) * K2[i];
  return R;
}
// Rotation matrix of a unit quaternion (w, x, y, z).
template <class T> static M3<T> quat_to_R(const T* qt) {
  T w = qt[0], x = qt[1], y = qt[2], z = qt[3];
  return M3<T>{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
               2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
               2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
}

template <class T> static V6<T> m6_v(const M6<T>& A, const V6<T>& x) {
  V6<T> y{};
  for (int i = 0; i < 6; ++i) {
    T s = 0;
    for (int k = 0; k < 6; ++k) s += A[i * 6 + k] * x[k];
    y[i] = s;
  }
  return y;
}
template <class T> static V6<T> m6T_v(const M6<T>& A, const V6<T>& x) {
  V6<T> y{};
  for (int i = 0; i < 6; ++i) {
    T s = 0;
    for (int k = 0; k < 6; ++k) s += A[k * 6 + i] * x[k];
    y[i] = s;
  }
  return y;
}
template <class T> static M6<T> m6_mul(const M6<T>& A, const M6<T>& B) {
  M6<T> C{};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T s = 0;
      for (int k = 0; k < 6; ++k) s += A[i * 6 + k] * B[k * 6 + j];
      C[i * 6 + j] = s;
    }
  return C;
}
template <class T> static M6<T> m6_T(const M6<T>& A) {
  M6<T> C{};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C[i * 6 + j] = A[j * 6 + i];
  return C;
}
// X^T A X : congruence used to carry an inertia from a child body to its parent.
template <class T> static M6<T> congruence(const M6<T>& X, const M6<T>& A) {
  return m6_mul(m6_T(X), m6_mul(A, X));
}

// Plucker motion transform from frame A to frame B, where E rotates
// A-coordinates into B-coordinates and r is B's origin in A-coordinates:
// X = [[E, 0], [-E r^x, E]].
template <class T> static M6<T> plucker(const M3<T>& E, const V3<T>& r) {
  M6<T> X{};
  M3<T> Erx = m3_mul(E, skew(r));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      X[i * 6 + j] = E[i * 3 + j];
      X[(i + 3) * 6 + (j + 3)] = E[i * 3 + j];
      X[(i + 3) * 6 + j] = -Erx[i * 3 + j];
    }
  return X;
}
// Motion cross product matrix  crm(v) = [[w^x, 0], [v^x, w^x]].
template <class T> static M6<T> crm(const V6<T>& v) {
  M6<T> C{};
  M3<T> wx = skew(V3<T>{v[0], v[1], v[2]}), vx = skew(V3<T>{v[3], v[4], v[5]});
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      C[i * 6 + j] = wx[i * 3 + j];
      C[(i + 3) * 6 + (j + 3)] = wx[i * 3 + j];
      C[(i + 3) * 6 + j] = vx[i * 3 + j];
    }
  return C;
}
// Force cross product: crf(v) = -crm(v)^T.
template <class T> static M6<T> crf(const V6<T>& v) {
  M6<T> C = crm(v), D{};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) D[i * 6 + j] = -C[j * 6 + i];
  return D;
}
// Spatial inertia of a rigid body of mass m, centre of mass c and rotational
// inertia Ic about c:  [[Ic + m c^x c^xT, m c^x], [m c^xT, m 1]].
template <class T> static M6<T> spatial_inertia(T m, const V3<T>& c, const M3<T>& Ic) {
  M6<T> I{};
  M3<T> cx = skew(c), cxT = m3_T(cx), ccT = m3_mul(cx, cxT);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      I[i * 6 + j] = Ic[i * 3 + j] + m * ccT[i * 3 + j];
      I[i * 6 + j + 3] = m * cx[i * 3 + j];
      I[(i + 3) * 6 + j] = m * cxT[i * 3 + j];
      I[(i + 3) * 6 + j + 3] = (i == j) ? m : T(0);
    }
  return I;
}

// Solve A x = b (n x n) by Gaussian elimination with partial pivoting.
template <class T> static std::vector<T> solve(std::vector<T> A, std::vector<T> b, int n) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
    if (piv != col) {
      for (int k = 0; k < n; ++k) std::swap(A[col * n + k], A[piv * n + k]);
      std::swap(b[col], b[piv]);
    }
    for (int r = col + 1; r < n; ++r) {
      T f = A[r * n + col] / A[col * n + col];
      for (int k = col; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
      b[r] -= f * b[col];
    }
  }
  std::vector<T> x(n);
  for (int r = n - 1; r >= 0; --r) {
    T s = b[r];
    for (int k = r + 1; k < n; ++k) s -= A[r * n + k] * x[k];
    x[r] = s / A[r * n + r];
  }
  return x;
}

// ---------------------------------------------------------------------------
// Model
// ---------------------------------------------------------------------------
template <class T> struct Model {
  int nb = 0, fb = 0, nu = 0, nc = 0, nq = 0, nv = 0;
  std::vector<int> parent, joint;  // joint[i] = actuated joint index of body i, -1 for the base
  std::vector<V3<T>> axis, p_tree, com, cpos;
  std::vector<M3<T>> R_tree;
  std::vector<M6<T>> Ibody;  // spatial inertia in body coordinates
  std::vector<T> mass, qmin, qmax, taumax, kp, kd, arm;
  std::vector<int> cbody;
  T k = 0, d = 0, mu = 0, eps = 0, g = 0;
  int ee_body = -1;
  V3<T> ee_pos{};
  T total_mass = 0;
  int nsub = 1;
};

template <class T> static Model<T> load_model(const orc_model* m) {
  Model<T> M;
  M.nb = m->n_bodies;
  M.fb = m->floating_base ? 1 : 0;
  M.nu = M.nb - M.fb;
  M.nc = m->n_contacts;
  M.nq = M.fb ? 7 + M.nu : M.nu;
  M.nv = M.fb ? 6 + M.nu : M.nu;
  for (int i = 0; i < M.nb; ++i) {
    M.parent.push_back(m->parent[i]);
    M.joint.push_back((M.fb && i == 0) ? -1 : i - M.fb);
    V3<T> a, p, c;
    M3<T> R;
    for (int k = 0; k < 3; ++k) {
      a[k] = (T)m->axis[i * 3 + k];
      p[k] = (T)m->p_tree[i * 3 + k];
      c[k] = (T)m->com[i * 3 + k];
    }
    for (int k = 0; k < 9; ++k) R[k] = (T)m->R_tree[i * 9 + k];
    M.axis.push_back(a);
    M.p_tree.push_back(p);
    M.com.push_back(c);
    M.R_tree.push_back(R);
    T ms = (T)m->mass[i];
    M.mass.push_back(ms);
    M.total_mass += ms;
    const double* in = m->inertia + i * 6;
    M3<T> Ic{(T)in[0], (T)in[3], (T)in[4], (T)in[3], (T)in[1], (T)in[5], (T)in[4], (T)in[5], (T)in[2]};
    M.Ibody.push_back(spatial_inertia<T>(ms, c, Ic));
  }
  for (int j = 0; j < M.nu; ++j) {
    M.qmin.push_back((T)m->q_min[j]);
    M.qmax.push_back((T)m->q_max[j]);
    M.taumax.push_back((T)m->tau_max[j]);
    M.kp.push_back((T)m->kp[j]);
    M.kd.push_back((T)m->kd[j]);
    M.arm.push_back(m->armature ? (T)m->armature[j] : T(0));
  }
  for (int c = 0; c < M.nc; ++c) {
    M.cbody.push_back(m->contact_body[c]);
    M.cpos.push_back(V3<T>{(T)m->contact_pos[c * 3], (T)m->contact_pos[c * 3 + 1], (T)m->contact_pos[c * 3 + 2]});
  }
  M.k = (T)m->k_contact;
  M.d = (T)m->d_contact;
  M.mu = (T)m->mu;
  M.eps = (T)m->eps_fric;
  M.g = (T)m->gravity;
  M.ee_body = m->ee_body;
  M.ee_pos = V3<T>{(T)m->ee_pos[0], (T)m->ee_pos[1], (T)m->ee_pos[2]};
  M.nsub = m->n_substeps;
  return M;
}

static bool model_ok(const orc_model* m) {
  if (!m || m->n_bodies <= 0 || m->n_bodies > 64 || m->n_substeps < 1) return false;
  if (m->floating_base && m->parent[0] != -1) return false;
  for (int i = 0; i < m->n_bodies; ++i) {
    if (m->parent[i] >= i) return false;
    if (m->floating_base && i > 0 && m->parent[i] < 0) return false;
  }
  for (int c = 0; c < m->n_contacts; ++c)
    if (m->contact_body[c] < 0 || m->contact_body[c] >= m->n_bodies) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Kinematics: parent-to-body transforms, world poses, body twists and the
// velocity-product accelerations c_i = v_i x (S_i qd_i), all in body coordinates.
// ---------------------------------------------------------------------------
template <class T> struct Kin {
  std::vector<M6<T>> Xup;
  std::vector<M3<T>> Rw;
  std::vector<V3<T>> pw;
  std::vector<V6<T>> vb, cb;
  std::vector<V6<T>> beta;  // body acceleration at qdd = 0 without gravity (velocity products)
  V6<T> ag_root{};  // gravity as a spatial acceleration: base coordinates (floating) or world
};

template <class T> static V6<T> joint_S(const Model<T>& M, int i) {
  return V6<T>{M.axis[i][0], M.axis[i][1], M.axis[i][2], 0, 0, 0};
}

template <class T> static Kin<T> kinematics(const Model<T>& M, const T* q, const T* v) {
  Kin<T> K;
  K.Xup.resize(M.nb);
  K.Rw.resize(M.nb);
  K.pw.resize(M.nb);
  K.vb.resize(M.nb);
  K.cb.resize(M.nb);
  K.beta.assign(M.nb, V6<T>{});
  const int qo = M.fb ? 7 : 0, vo = M.fb ? 6 : 0;
  V3<T> gw{0, 0, -M.g};
  for (int i = 0; i < M.nb; ++i) {
    if (M.fb && i == 0) {
      K.Rw[0] = quat_to_R(q + 3);
      K.pw[0] = V3<T>{q[0], q[1], q[2]};
      for (int k = 0; k < 6; ++k) K.vb[0][k] = v[k];
      K.cb[0] = V6<T>{};
      V3<T> gb = m3_v(m3_T(K.Rw[0]), gw);
      K.ag_root = V6<T>{0, 0, 0, gb[0], gb[1], gb[2]};
      continue;
    }
    int j = M.joint[i], lam = M.parent[i];
    T qi = q[qo + j], qdi = v[vo + j];
    M3<T> C = m3_mul(M.R_tree[i], rot_axis(M.axis[i], qi));  // body i in parent frame
    K.Xup[i] = plucker(m3_T(C), M.p_tree[i]);
    V6<T> vpar{};
    if (lam >= 0) {
      K.Rw[i] = m3_mul(K.Rw[lam], C);
      V3<T> off = m3_v(K.Rw[lam], M.p_tree[i]);
      for (int k = 0; k < 3; ++k) K.pw[i][k] = K.pw[lam][k] + off[k];
      vpar = K.vb[lam];
    } else {
      K.Rw[i] = C;
      K.pw[i] = M.p_tree[i];
    }
    V6<T> S = joint_S(M, i), vJ{};
    for (int k = 0; k < 6; ++k) vJ[k] = S[k] * qdi;
    V6<T> xv = m6_v(K.Xup[i], vpar);
    for (int k = 0; k < 6; ++k) K.vb[i][k] = xv[k] + vJ[k];
    K.cb[i] = m6_v(crm(K.vb[i]), vJ);
    V6<T> xb = m6_v(K.Xup[i], lam >= 0 ? K.beta[lam] : V6<T>{});
    for (int k = 0; k < 6; ++k) K.beta[i][k] = xb[k] + K.cb[i][k];
  }
  if (!M.fb) K.ag_root = V6<T>{0, 0, 0, gw[0], gw[1], gw[2]};
  return K;
}

// ---------------------------------------------------------------------------
// Soft contact: penalty spring-damper normal force on ground z = 0 (no
// adhesion) and Coulomb friction smoothed by eps.  Forces become spatial
// forces on the carrying body, in body coordinates.
// ---------------------------------------------------------------------------
template <class T> struct ContactOut {
  std::vector<V3<T>> pos, vel, force;
  std::vector<int> active;  // f_n > 0
  uint32_t mask = 0;
};

// Linearly implicit treatment (step dt_imp > 0): the contact force is taken at
// the end-of-step point velocity v_c + dt J_c qdd.  Its velocity Jacobian D
// (normal: d; tangential: mu f_n (I - v_t v_t^T / n^2) / n with
// n = sqrt(|v_t|^2 + eps^2); the tangential-normal coupling is dropped so D is
// symmetric) then acts on J_c qdd like an added mass dt P^T D P on the body,
// with P = [-r^x, 1] the point-velocity map in body coordinates.
template <class T>
static ContactOut<T> contacts(const Model<T>& M, const Kin<T>& K, std::vector<V6<T>>& fext, T dt_imp = 0,
                              std::vector<M6<T>>* Iadd = nullptr) {
  ContactOut<T> C;
  fext.assign(M.nb, V6<T>{});
  if (Iadd) Iadd->assign(M.nb, M6<T>{});
  for (int c = 0; c < M.nc; ++c) {
    int b = M.cbody[c];
    const V3<T>& r = M.cpos[c];
    V3<T> pr = m3_v(K.Rw[b], r), p{};
    for (int k = 0; k < 3; ++k) p[k] = K.pw[b][k] + pr[k];
    V3<T> w{K.vb[b][0], K.vb[b][1], K.vb[b][2]}, vo{K.vb[b][3], K.vb[b][4], K.vb[b][5]};
    V3<T> wr = cross(w, r), vl{};
    for (int k = 0; k < 3; ++k) vl[k] = vo[k] + wr[k];
    V3<T> vw = m3_v(K.Rw[b], vl);
    T fn = 0;
    if (p[2] < 0) fn = std::max(T(0), -M.k * p[2] - M.d * vw[2]);
    T nrm = std::sqrt(vw[0] * vw[0] + vw[1] * vw[1] + M.eps * M.eps);
    V3<T> f{-M.mu * fn * vw[0] / nrm, -M.mu * fn * vw[1] / nrm, fn};
    V3<T> fb = m3_v(m3_T(K.Rw[b]), f);
    V3<T> tb = cross(r, fb);
    for (int k = 0; k < 3; ++k) {
      fext[b][k] += tb[k];
      fext[b][k + 3] += fb[k];
    }
    if (Iadd && dt_imp > 0 && fn > 0) {
      M3<T> Dw{};
      T a = M.mu * fn / nrm, n2 = nrm * nrm;
      Dw[0] = a * (1 - vw[0] * vw[0] / n2);
      Dw[1] = a * (-vw[0] * vw[1] / n2);
      Dw[3] = Dw[1];
      Dw[4] = a * (1 - vw[1] * vw[1] / n2);
      Dw[8] = M.d;
      M3<T> Db = m3_mul(m3_T(K.Rw[b]), m3_mul(Dw, K.Rw[b]));
      // P = [-r^x, 1] (3 x 6); added inertia dt P^T Db P
      M3<T> rx = skew(r);
      T P[3][6];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          P[i][j] = -rx[i * 3 + j];
          P[i][j + 3] = (i == j) ? T(1) : T(0);
        }
      M6<T>& A = (*Iadd)[b];
      for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
          T sacc = 0;
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) sacc += P[k][i] * Db[k * 3 + l] * P[l][j];
          A[i * 6 + j] += dt_imp * sacc;
        }
    }
    C.pos.push_back(p);
    C.vel.push_back(vw);
    C.force.push_back(f);
    C.active.push_back(fn > 0 ? 1 : 0);
    if (fn > 0 && c < 32) C.mask |= (1u << c);
  }
  return C;
}

// PD tracking law (eq. pd-controller) with torques clipped to the actuator
// limits.  With a step dt_imp > 0 the law is linearly implicit in the joint
// velocity: an unsaturated joint also carries the gain g = dt (Kd + dt Kp), so
// the applied torque is tau - g qdd (the PD evaluated at v + dt qdd and at
// q + dt (v + dt qdd)); a saturated joint carries g = 0.
template <class T> struct PDOut {
  std::vector<T> tau, g;
};
template <class T>
static PDOut<T> pd_law(const Model<T>& M, const T* q, const T* v, const T* qr, const T* vr, T dt_imp) {
  PDOut<T> o;
  o.tau.resize(M.nu);
  o.g.assign(M.nu, 0);
  const int qo = M.fb ? 7 : 0, vo = M.fb ? 6 : 0;
  for (int j = 0; j < M.nu; ++j) {
    T t = M.kp[j] * (qr[j] - q[qo + j]) + M.kd[j] * (vr[j] - v[vo + j]);
    if (t >= M.taumax[j]) {
      o.tau[j] = M.taumax[j];
    } else if (t <= -M.taumax[j]) {
      o.tau[j] = -M.taumax[j];
    } else {
      o.tau[j] = t;
      o.g[j] = dt_imp * (M.kd[j] + dt_imp * M.kp[j]);
    }
  }
  return o;
}

// ---------------------------------------------------------------------------
// Articulated-body algorithm (Featherstone, RBDA ch. 7, floating base ch. 9),
// body coordinates.  Gravity enters by shifting every acceleration by -a_g.
// Returns qdd: [base spatial acceleration (6, base coordinates), joints] or
// [joints] for a fixed base.
// ---------------------------------------------------------------------------
// Optional implicit terms: Iadd[i] is an added inertia acting on the part
// J_i qdd of body i's acceleration (so its bias uses a_g - beta_i), and g[j]
// is a joint gain acting on qdd_j.
template <class T>
static std::vector<T> aba(const Model<T>& M, const Kin<T>& K, const T* tau, const std::vector<V6<T>>& fext,
                          const std::vector<M6<T>>* Iadd = nullptr, const T* g = nullptr) {
  const int nb = M.nb;
  std::vector<M6<T>> IA(nb);
  std::vector<V6<T>> pA(nb), U(nb), a(nb);
  std::vector<T> D(nb, 1), u(nb, 0);
  V3<T> gw{0, 0, -M.g};
  for (int i = 0; i < nb; ++i) {
    IA[i] = M.Ibody[i];
    V6<T> h = m6_v(M.Ibody[i], K.vb[i]);
    V6<T> b = m6_v(crf(K.vb[i]), h);
    for (int k = 0; k < 6; ++k) pA[i][k] = b[k] - fext[i][k];
    if (Iadd) {
      const M6<T>& A = (*Iadd)[i];
      V3<T> gb = m3_v(m3_T(K.Rw[i]), gw);
      V6<T> sh{-K.beta[i][0], -K.beta[i][1], -K.beta[i][2], gb[0] - K.beta[i][3], gb[1] - K.beta[i][4],
               gb[2] - K.beta[i][5]};
      V6<T> Ash = m6_v(A, sh);
      for (int k = 0; k < 36; ++k) IA[i][k] += A[k];
      for (int k = 0; k < 6; ++k) pA[i][k] += Ash[k];
    }
  }
  for (int i = nb - 1; i >= M.fb; --i) {
    V6<T> S = joint_S(M, i);
    U[i] = m6_v(IA[i], S);
    T Dv = 0, sp = 0;
    for (int k = 0; k < 6; ++k) {
      Dv += S[k] * U[i][k];
      sp += S[k] * pA[i][k];
    }
    D[i] = Dv + M.arm[M.joint[i]] + (g ? g[M.joint[i]] : T(0));
    u[i] = tau[M.joint[i]] - sp;
    int lam = M.parent[i];
    if (lam >= 0) {
      M6<T> Ia = IA[i];
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) Ia[r * 6 + c] -= U[i][r] * U[i][c] / D[i];
      V6<T> Iac = m6_v(Ia, K.cb[i]), pa{};
      for (int k = 0; k < 6; ++k) pa[k] = pA[i][k] + Iac[k] + U[i][k] * u[i] / D[i];
      M6<T> Ip = congruence(K.Xup[i], Ia);
      V6<T> pp = m6T_v(K.Xup[i], pa);
      for (int k = 0; k < 36; ++k) IA[lam][k] += Ip[k];
      for (int k = 0; k < 6; ++k) pA[lam][k] += pp[k];
    }
  }
  std::vector<T> qdd(M.nv, 0);
  V6<T> a_world{};  // shifted acceleration of the fixed world: -a_g
  for (int k = 0; k < 6; ++k) a_world[k] = -K.ag_root[k];
  if (M.fb) {
    std::vector<T> A(IA[0].begin(), IA[0].end()), b(6);
    for (int k = 0; k < 6; ++k) b[k] = -pA[0][k];
    std::vector<T> x = solve(A, b, 6);
    for (int k = 0; k < 6; ++k) a[0][k] = x[k];
    for (int k = 0; k < 6; ++k) qdd[k] = a[0][k] + K.ag_root[k];
  }
  for (int i = M.fb; i < nb; ++i) {
    int lam = M.parent[i];
    V6<T> ap = m6_v(K.Xup[i], lam >= 0 ? a[lam] : a_world);
    for (int k = 0; k < 6; ++k) a[i][k] = ap[k] + K.cb[i][k];
    V6<T> S = joint_S(M, i);
    T Ua = 0;
    for (int k = 0; k < 6; ++k) Ua += U[i][k] * a[i][k];
    T qddi = (u[i] - Ua) / D[i];
    for (int k = 0; k < 6; ++k) a[i][k] += S[k] * qddi;
    qdd[(M.fb ? 6 : 0) + M.joint[i]] = qddi;
  }
  return qdd;
}

// Composite-rigid-body algorithm: joint-space inertia matrix M(q) (nv x nv).
template <class T> static std::vector<T> crba(const Model<T>& M, const Kin<T>& K) {
  const int nb = M.nb, nv = M.nv, vo = M.fb ? 6 : 0;
  std::vector<M6<T>> IC(M.Ibody);
  for (int i = nb - 1; i >= 0; --i) {
    int lam = M.parent[i];
    if (lam >= 0 && !(M.fb && i == 0)) {
      M6<T> Ip = congruence(K.Xup[i], IC[i]);
      for (int k = 0; k < 36; ++k) IC[lam][k] += Ip[k];
    }
  }
  std::vector<T> H(nv * nv, 0);
  if (M.fb)
    for (int r = 0; r < 6; ++r)
      for (int c = 0; c < 6; ++c) H[r * nv + c] = IC[0][r * 6 + c];
  for (int i = M.fb; i < nb; ++i) {
    int di = vo + M.joint[i];
    V6<T> S = joint_S(M, i);
    V6<T> F = m6_v(IC[i], S);
    T hii = 0;
    for (int k = 0; k < 6; ++k) hii += S[k] * F[k];
    H[di * nv + di] = hii + M.arm[M.joint[i]];
    int j = i;
    while (M.parent[j] >= 0) {
      F = m6T_v(K.Xup[j], F);
      j = M.parent[j];
      if (M.fb && j == 0) {
        for (int k = 0; k < 6; ++k) {
          H[k * nv + di] = F[k];
          H[di * nv + k] = F[k];
        }
      } else {
        int dj = vo + M.joint[j];
        V6<T> Sj = joint_S(M, j);
        T hij = 0;
        for (int k = 0; k < 6; ++k) hij += Sj[k] * F[k];
        H[di * nv + dj] = hij;
        H[dj * nv + di] = hij;
      }
    }
  }
  return H;
}

// Recursive Newton-Euler inverse dynamics: generalised forces that produce qdd
// (base part = net spatial force the base would need; zero for a free base).
template <class T>
static std::vector<T> rnea(const Model<T>& M, const Kin<T>& K, const T* qdd, const std::vector<V6<T>>& fext) {
  const int nb = M.nb, vo = M.fb ? 6 : 0;
  std::vector<V6<T>> a(nb), f(nb);
  V6<T> a_world{};
  for (int k = 0; k < 6; ++k) a_world[k] = -K.ag_root[k];
  for (int i = 0; i < nb; ++i) {
    if (M.fb && i == 0) {
      for (int k = 0; k < 6; ++k) a[0][k] = qdd[k] - K.ag_root[k];
    } else {
      int lam = M.parent[i];
      V6<T> ap = m6_v(K.Xup[i], lam >= 0 ? a[lam] : a_world);
      V6<T> S = joint_S(M, i);
      T qddi = qdd[vo + M.joint[i]];
      for (int k = 0; k < 6; ++k) a[i][k] = ap[k] + S[k] * qddi + K.cb[i][k];
    }
    V6<T> Ia = m6_v(M.Ibody[i], a[i]);
    V6<T> h = m6_v(M.Ibody[i], K.vb[i]);
    V6<T> b = m6_v(crf(K.vb[i]), h);
    for (int k = 0; k < 6; ++k) f[i][k] = Ia[k] + b[k] - fext[i][k];
  }
  std::vector<T> tau(M.nv, 0);
  for (int i = nb - 1; i >= 0; --i) {
    if (M.fb && i == 0) {
      for (int k = 0; k < 6; ++k) tau[k] = f[0][k];
      continue;
    }
    V6<T> S = joint_S(M, i);
    T t = 0;
    for (int k = 0; k < 6; ++k) t += S[k] * f[i][k];
    tau[vo + M.joint[i]] = t + M.arm[M.joint[i]] * qdd[vo + M.joint[i]];
    int lam = M.parent[i];
    if (lam >= 0) {
      V6<T> fp = m6T_v(K.Xup[i], f[i]);
      for (int k = 0; k < 6; ++k) f[lam][k] += fp[k];
    }
  }
  return tau;
}

// ---------------------------------------------------------------------------
// Cubic Hermite segment (Sec. III-A, eq. hermite_segment and its basis):
// position and its time derivative at step h of a horizon of H steps whose
// N_k knots are spread uniformly over H*dt.  The segment and local time come
// from integer arithmetic: m = h (N_k-1), seg = min(m / H, N_k-2),
// s = (m - seg H) / H.
// ---------------------------------------------------------------------------
template <class T>
static void hermite_eval(const T* knots, int nk, int nu, int H, T delta, int h, int j, T* qr, T* vr) {
  long m = (long)h * (nk - 1);
  int seg = (int)std::min<long>(m / H, nk - 2);
  T s = (T)(m - (long)seg * H) / (T)H;
  T s2 = s * s, s3 = s2 * s;
  T h00 = 2 * s3 - 3 * s2 + 1, h10 = s3 - 2 * s2 + s, h01 = -2 * s3 + 3 * s2, h11 = s3 - s2;
  T d00 = 6 * s2 - 6 * s, d10 = 3 * s2 - 4 * s + 1, d01 = -6 * s2 + 6 * s, d11 = 3 * s2 - 2 * s;
  const T* Q = knots;
  const T* V = knots + nk * nu;
  T q0 = Q[seg * nu + j], q1 = Q[(seg + 1) * nu + j];
  T v0 = V[seg * nu + j], v1 = V[(seg + 1) * nu + j];
  *qr = h00 * q0 + h10 * delta * v0 + h01 * q1 + h11 * delta * v1;
  *vr = (d00 * q0 + d10 * delta * v0 + d01 * q1 + d11 * delta * v1) / delta;
}

// Hermite interpolant at an arbitrary time t in [0, H dt] (used only for the
// dense-route check: resampling a dense weighted average at node times).
template <class T>
static void hermite_at_time(const T* knots, int nk, int nu, T delta, T t, int j, T* qr, T* vr) {
  int seg = (int)std::floor(t / delta);
  seg = std::max(0, std::min(seg, nk - 2));
  T s = (t - seg * delta) / delta;
  T s2 = s * s, s3 = s2 * s;
  T h00 = 2 * s3 - 3 * s2 + 1, h10 = s3 - 2 * s2 + s, h01 = -2 * s3 + 3 * s2, h11 = s3 - s2;
  T d00 = 6 * s2 - 6 * s, d10 = 3 * s2 - 4 * s + 1, d01 = -6 * s2 + 6 * s, d11 = 3 * s2 - 2 * s;
  const T* Q = knots;
  const T* V = knots + nk * nu;
  T q0 = Q[seg * nu + j], q1 = Q[(seg + 1) * nu + j];
  T v0 = V[seg * nu + j], v1 = V[(seg + 1) * nu + j];
  *qr = h00 * q0 + h10 * delta * v0 + h01 * q1 + h11 * delta * v1;
  *vr = (d00 * q0 + d10 * delta * v0 + d01 * q1 + d11 * delta * v1) / delta;
}

// ---------------------------------------------------------------------------
// Noise schedule (Sec. III-B).  Exponential mode: the isotropic kernel of eq.
// overall-noise-kernel read as a standard deviation multiplier,
// sigma[iota][k] = scale_q * exp(-iota/(beta1 I) - (N_k - k)/(beta2 N_k)),
// iota = I - i.  Linear mode: sigma[k] = lo + (hi - lo) k/(N_k - 1) for every
// iteration.  The velocity standard deviation is sigma / Delta.
// ---------------------------------------------------------------------------
static void sigma_table(const orc_params* p, double* sig) {
  const int I = p->n_iters, K = p->n_knots;
  for (int it = 0; it < I; ++it)
    for (int k = 0; k < K; ++k) {
      double s;
      if (p->noise_mode == 0)
        s = p->scale_q * std::exp(-(double)it / (p->beta1 * I) - (double)(K - k) / (p->beta2 * K));
      else
        s = p->sigma_lo + (p->sigma_hi - p->sigma_lo) * (double)k / (double)(K - 1);
      sig[it * K + k] = s;
    }
}

// Perturbed, clipped and derivative-clamped knots of sample n (Alg. 1 sampling
// step; eq. vel-clamp with the distance to the nearest bound over Delta/2).
// Sample 0 is the nominal itself, clipped and clamped the same way.
// Spline variants of the ablation (Sec. V, splines; the paper's comparison of
// cubic Hermite splines with position-only cubic and quadratic splines whose
// velocity targets are zero).  The position-only variants sample only the
// position knots; their knot slopes (dq/dt) are derived from the positions and
// kept in the velocity block, and the curve is evaluated in Hermite form:
//   mode 1, natural cubic spline: C2 at the interior knots and zero second
//     derivative at both ends, i.e. m_{k-1} + 4 m_k + m_{k+1} = 3 (q_{k+1} - q_{k-1}) / Delta,
//     2 m_0 + m_1 = 3 (q_1 - q_0) / Delta, m_{K-2} + 2 m_{K-1} = 3 (q_{K-1} - q_{K-2}) / Delta
//     (a cubic spline is the Hermite spline of its own knot slopes);
//   mode 2, quadratic spline: C1 pieces q_k + m_k tau + c tau^2 with zero initial
//     slope, m_0 = 0, m_{k+1} = 2 (q_{k+1} - q_k) / Delta - m_k (a quadratic
//     piece is the Hermite cubic of its end values and slopes).
template <class T> static void position_spline_slopes(int mode, int K, int nu, T delta, T* knots) {
  const T* Q = knots;
  T* V = knots + K * nu;
  for (int j = 0; j < nu; ++j) {
    if (mode == 2) {
      V[j] = 0;
      for (int k = 0; k + 1 < K; ++k) V[(k + 1) * nu + j] = 2 * (Q[(k + 1) * nu + j] - Q[k * nu + j]) / delta - V[k * nu + j];
      continue;
    }
    // mode 1: tridiagonal system (sub/super diagonal 1), Thomas elimination
    std::vector<T> diag(K), rhs(K);
    for (int k = 0; k < K; ++k) {
      const bool end = k == 0 || k == K - 1;
      diag[k] = end ? T(2) : T(4);
      const T qa = Q[(k == 0 ? 0 : k - 1) * nu + j], qb = Q[(k == K - 1 ? K - 1 : k + 1) * nu + j];
      rhs[k] = 3 * (qb - qa) / delta;
    }
    for (int k = 1; k < K; ++k) {
      const T w = T(1) / diag[k - 1];
      diag[k] -= w;
      rhs[k] -= w * rhs[k - 1];
    }
    V[(K - 1) * nu + j] = rhs[K - 1] / diag[K - 1];
    for (int k = K - 2; k >= 0; --k) V[k * nu + j] = (rhs[k] - V[(k + 1) * nu + j]) / diag[k];
  }
}

template <class T>
static void sample_knots(const Model<T>& M, const orc_params* p, const T* nominal, const double* sig,
                         uint64_t seed, uint32_t tick, int iota, int n, T* out) {
  const int K = p->n_knots, nu = M.nu;
  const T delta = (T)(p->horizon * p->dt / (K - 1));
  for (int k = 0; k < K; ++k)
    for (int j = 0; j < nu; ++j) {
      int m = k * nu + j;
      T zq = 0, zv = 0;
      if (n > 0) knot_normals<T>(seed, tick, iota, n, m, &zq, &zv);
      T sq = (T)sig[iota * K + k];
      T sv = sq / delta;
      T tq = nominal[m] + sq * zq;
      tq = std::min(std::max(tq, M.qmin[j]), M.qmax[j]);
      T lim = 2 * std::min(M.qmax[j] - tq, tq - M.qmin[j]) / delta;
      T tv = nominal[K * nu + m] + sv * zv;
      tv = std::min(std::max(tv, -lim), lim);
      out[m] = tq;
      out[K * nu + m] = tv;
    }
  if (p->spline_mode != 0) position_spline_slopes<T>(p->spline_mode, K, nu, delta, out);
}

// ---------------------------------------------------------------------------
// One rollout: PD tracking of the Hermite reference (eq. pd-controller, torques
// clipped), soft contact, ABA, running cost on the pre-step state, semi-implicit
// Euler; terminal cost on x_H (Sec. IV-A cost terms).
// ---------------------------------------------------------------------------
template <class T> struct RolloutDebug {
  T* traj = nullptr;        // [(H+1)][nq+nv]
  uint32_t* masks = nullptr;  // [H]
  T* stage = nullptr;       // [H+1]
};

template <class T> static T orientation_angle(const T* quat) {
  T vn = std::sqrt(quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
  return 2 * std::atan2(vn, std::fabs(quat[0]));
}

// ||log3(R_base^T R_des)||: the rotation angle of the relative rotation, i.e. of
// the quaternion conj(q_base) * q_des (Sec. IV-A, orientation residual); an
// all-zero target stands for the identity.
template <class T> static T orientation_error(const T* qb, const double* qd) {
  const bool id = qd[0] == 0 && qd[1] == 0 && qd[2] == 0 && qd[3] == 0;
  const T d0 = id ? T(1) : (T)qd[0], d1 = id ? T(0) : (T)qd[1], d2 = id ? T(0) : (T)qd[2], d3 = id ? T(0) : (T)qd[3];
  // conj(qb) = (w, -x, -y, -z); Hamilton product with (d0, d1, d2, d3)
  const T r[4] = {qb[0] * d0 + qb[1] * d1 + qb[2] * d2 + qb[3] * d3,
                  qb[0] * d1 - qb[1] * d0 - qb[2] * d3 + qb[3] * d2,
                  qb[0] * d2 + qb[1] * d3 - qb[2] * d0 - qb[3] * d1,
                  qb[0] * d3 - qb[1] * d2 + qb[2] * d1 - qb[3] * d0};
  return orientation_angle(r);
}

template <class T> static V3<T> point_world(const Kin<T>& K, int b, const V3<T>& r) {
  V3<T> pr = m3_v(K.Rw[b], r), p{};
  for (int k = 0; k < 3; ++k) p[k] = K.pw[b][k] + pr[k];
  return p;
}

template <class T>
static void integrate(const Model<T>& M, T dt, T* q, T* v, const std::vector<T>& qdd) {
  for (int k = 0; k < M.nv; ++k) v[k] += dt * qdd[k];
  const int qo = M.fb ? 7 : 0, vo = M.fb ? 6 : 0;
  for (int j = 0; j < M.nu; ++j) q[qo + j] += dt * v[vo + j];
  if (M.fb) {
    M3<T> R = quat_to_R(q + 3);
    V3<T> dp = m3_v(R, V3<T>{v[3], v[4], v[5]});
    for (int k = 0; k < 3; ++k) q[k] += dt * dp[k];
    T wn = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    T e[4] = {1, 0, 0, 0};
    if (wn > 0) {
      T th = wn * dt / 2, sn = std::sin(th) / wn;
      e[0] = std::cos(th);
      e[1] = sn * v[0];
      e[2] = sn * v[1];
      e[3] = sn * v[2];
    }
    T a0 = q[3], a1 = q[4], a2 = q[5], a3 = q[6];
    T r0 = a0 * e[0] - a1 * e[1] - a2 * e[2] - a3 * e[3];
    T r1 = a0 * e[1] + a1 * e[0] + a2 * e[3] - a3 * e[2];
    T r2 = a0 * e[2] - a1 * e[3] + a2 * e[0] + a3 * e[1];
    T r3 = a0 * e[3] + a1 * e[2] - a2 * e[1] + a3 * e[0];
    T nn = std::sqrt(r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
    q[3] = r0 / nn;
    q[4] = r1 / nn;
    q[5] = r2 / nn;
    q[6] = r3 / nn;
  }
}

// One control step h of a rollout, advancing (q, v) in place: n_sub physics
// substeps of dt / n_sub (linearly implicit Euler: ABA with the implicit PD and
// contact terms, then v += dt qdd, q += dt v), the PD law tracking the spline at
// every substep time.  Returns the running cost of the step, taken on the state,
// the clipped PD torques and the contact forces of its first substep.  Optional
// outputs of that first substep: the contact-activity mask, the accelerations
// qdd0 [nv] and the normal force of every contact point fn0 [nc].
template <class T>
static T control_step(const Model<T>& M, const orc_params* p, const T* knots, int h, T* q, T* v,
                      uint32_t* mask = nullptr, T* qdd0 = nullptr, T* fn0 = nullptr) {
  const int H = p->horizon, K = p->n_knots, nu = M.nu, ns = M.nsub;
  const int F = H * ns;
  const T dtf = (T)(p->dt / ns), delta = (T)(p->horizon * p->dt / (K - 1));
  const int qo = M.fb ? 7 : 0;
  std::vector<T> tau(nu), qref(nu), vref(nu);
  std::vector<V6<T>> fext;
  std::vector<M6<T>> Iadd;
  T c = 0;
  for (int sub = 0; sub < ns; ++sub) {
    const int f = h * ns + sub;
    const bool control = sub == 0;
    for (int j = 0; j < nu; ++j) {
      hermite_eval(knots, K, nu, F, delta, f, j, &qref[j], &vref[j]);
      if (p->spline_mode != 0) vref[j] = 0;  // position-only variants: zero velocity targets
    }
    PDOut<T> pd = pd_law(M, q, v, qref.data(), vref.data(), dtf);
    tau = pd.tau;
    Kin<T> Kn = kinematics(M, q, v);
    ContactOut<T> C = contacts(M, Kn, fext, dtf, &Iadd);
    std::vector<T> qdd = aba(M, Kn, tau.data(), fext, &Iadd, pd.g.data());
    if (control) {
      T eff = 0;
      for (int j = 0; j < nu; ++j) eff += tau[j] * tau[j];
      if (p->cost_kind == 0) {
        V3<T> ee = point_world(Kn, M.ee_body, M.ee_pos);
        T dz = ee[2] - (T)p->z_des;
        c = (T)p->w_ee * dz * dz + (T)p->w_tau * eff;
      } else {
        T phi = orientation_error(q + 3, p->q_des);
        T dq2 = 0;
        for (int j = 0; j < nu; ++j) {
          T e = q[qo + j] - (T)p->q0_cost[j];
          dq2 += e * e;
        }
        T cv = 0, cf = 0;
        for (int ci = 0; ci < M.nc; ++ci) {
          if (C.active[ci]) cv += std::fabs(C.vel[ci][0]) + std::fabs(C.vel[ci][1]) + std::fabs(C.vel[ci][2]);
          cf += std::fabs(C.force[ci][0]) + std::fabs(C.force[ci][1]) + std::fabs(C.force[ci][2] - (T)p->f0z[ci]);
        }
        c = (T)p->w_h * std::fabs(q[2] - (T)p->z_des) + (T)p->w_or * phi * phi + (T)p->w_q * dq2 +
            (T)p->w_cv * cv + (T)p->w_cf * cf + (T)p->w_eff * eff;
      }
      if (mask) *mask = C.mask;
      if (qdd0) std::copy(qdd.begin(), qdd.end(), qdd0);
      if (fn0)
        for (int ci = 0; ci < M.nc; ++ci) fn0[ci] = C.force[ci][2];
    }
    integrate(M, dtf, q, v, qdd);
  }
  return c;
}

// Terminal cost on x_H (Sec. IV-A): the L1 distance of the base position to
// p(x0) + v_des H dt (its height z_terminal instead when terminal_z_abs), or
// for the end-effector task w_ee (z_ee - z_des)^2.
template <class T>
static T terminal_cost(const Model<T>& M, const orc_params* p, const T* x0, const T* q, const T* v) {
  T cT = 0;
  if (p->cost_kind == 0) {
    Kin<T> Kn = kinematics(M, q, v);
    V3<T> ee = point_world(Kn, M.ee_body, M.ee_pos);
    T dz = ee[2] - (T)p->z_des;
    cT = (T)p->w_ee * dz * dz;
  } else {
    T Th = (T)(p->horizon * p->dt);
    for (int k = 0; k < 3; ++k) {
      const T target = (k == 2 && p->terminal_z_abs) ? (T)p->z_terminal : x0[k] + (T)p->v_des[k] * Th;
      cT += std::fabs(q[k] - target);
    }
    cT *= (T)p->w_H;
  }
  return cT;
}

// One rollout (Alg. 1 simulate step): H control steps from x0, the running
// costs summed as they come (no dt factor), then the terminal cost; a
// non-finite total becomes +inf.
template <class T>
static T rollout(const Model<T>& M, const orc_params* p, const T* x0, const T* knots, RolloutDebug<T> dbg) {
  const int H = p->horizon, nq = M.nq, nv = M.nv;
  std::vector<T> q(x0, x0 + nq), v(x0 + nq, x0 + nq + nv);
  T S = 0;
  for (int h = 0; h < H; ++h) {
    if (dbg.traj)
      for (int k = 0; k < nq + nv; ++k) dbg.traj[h * (nq + nv) + k] = k < nq ? q[k] : v[k - nq];
    uint32_t mk = 0;
    const T c = control_step(M, p, knots, h, q.data(), v.data(), &mk);
    if (dbg.masks) dbg.masks[h] = mk;
    if (dbg.stage) dbg.stage[h] = c;
    S += c;
  }
  if (dbg.traj)
    for (int k = 0; k < nq + nv; ++k) dbg.traj[H * (nq + nv) + k] = k < nq ? q[k] : v[k - nq];
  const T cT = terminal_cost(M, p, x0, q.data(), v.data());
  if (dbg.stage) dbg.stage[H] = cT;
  S += cT;
  if (!std::isfinite((double)S)) S = std::numeric_limits<T>::infinity();
  return S;
}

// ---------------------------------------------------------------------------
// Importance weights (eq. omega-weights, and the min-max normalised form of
// eq. softmax_minmax).  Non-finite costs get zero weight and are excluded from
// the minimum and maximum; a zero cost range gives uniform weights.  Returns
// the number of finite costs; *nstar = lowest index attaining the minimum.
// ---------------------------------------------------------------------------
static int weights(int n, const double* S, double lambda, int mode, double* w, int* nstar) {
  double smin = std::numeric_limits<double>::infinity(), smax = -smin;
  int nf = 0, arg = -1;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(S[i])) continue;
    ++nf;
    if (S[i] < smin) {
      smin = S[i];
      arg = i;
    }
    if (S[i] > smax) smax = S[i];
  }
  *nstar = arg;
  if (nf == 0) {
    for (int i = 0; i < n; ++i) w[i] = 0;
    return 0;
  }
  double range = smax - smin;
  double z = 0;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(S[i])) {
      w[i] = 0;
      continue;
    }
    double sh;
    if (mode == 0)
      sh = range > 0 ? (S[i] - smin) / range : 0.0;
    else
      sh = S[i] - smin;
    w[i] = std::exp(-sh / lambda);
    z += w[i];
  }
  for (int i = 0; i < n; ++i) w[i] /= z;
  return nf;
}

static bool params_ok(const orc_model* m, const orc_params* p) {
  if (!p || p->n_samples < 1 || p->horizon < 1 || p->n_knots < 2 || p->n_iters < 1) return false;
  if (!(p->dt > 0) || !(p->lambda > 0)) return false;
  if (p->cost_kind == 0 && (m->ee_body < 0 || m->ee_body >= m->n_bodies)) return false;
  if (p->cost_kind == 1 && !m->floating_base) return false;
  if (p->cost_kind == 1 && (!p->q0_cost || (m->n_contacts > 0 && !p->f0z))) return false;
  if (p->spline_mode < 0 || p->spline_mode > 2) return false;
  return true;
}

template <class T>
static void run_rollouts(const Model<T>& M, const orc_params* p, const double* x0d, const double* nominal_d,
                         uint64_t seed, uint32_t tick, int iota, int n0, int count, double* S_out,
                         double* samples_out, int threads) {
  const int E = 2 * p->n_knots * M.nu;
  std::vector<double> sig(p->n_iters * p->n_knots);
  sigma_table(p, sig.data());
  std::vector<T> x0(x0d, x0d + M.nq + M.nv), nominal(nominal_d, nominal_d + E);
#pragma omp parallel for schedule(dynamic) num_threads(threads)
  for (int i = 0; i < count; ++i) {
    std::vector<T> th(E);
    sample_knots(M, p, nominal.data(), sig.data(), seed, tick, iota, n0 + i, th.data());
    S_out[i] = (double)rollout(M, p, x0.data(), th.data(), RolloutDebug<T>{});
    if (samples_out)
      for (int e = 0; e < E; ++e) samples_out[(size_t)i * E + e] = (double)th[e];
  }
}

}  // namespace orc

using namespace orc;

extern "C" {

int orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
  return 0;
}

// Standard normals (z_q, z_v) of knot slots m = 0..count-1 for sample n.
int orc_normals(uint64_t seed, uint32_t tick, int iota, int n, int count, double* zq, double* zv) {
  for (int m = 0; m < count; ++m) knot_normals<double>(seed, tick, iota, n, m, zq + m, zv + m);
  return 0;
}

int orc_sigma_table(const orc_params* p, double* sig) {
  if (!p || p->n_iters < 1 || p->n_knots < 2) return -1;
  sigma_table(p, sig);
  return 0;
}

int orc_hermite(const double* knots, int nk, int nu, int H, double dt, int h, int j, double* qr, double* vr) {
  if (nk < 2 || H < 1 || h < 0 || h > H) return -1;
  double delta = H * dt / (nk - 1);
  hermite_eval<double>(knots, nk, nu, H, delta, h, j, qr, vr);
  return 0;
}

// Warm start (Sec. III-E, the shift of tau_best): the knots of the best
// trajectory moved forward by n_steps control steps, i.e. the old spline
// evaluated at t_k + n_steps dt, t_k = k Delta; past the end of the horizon the
// final action repeats, so the time is clamped to T = H dt.  Position and
// velocity knots are the spline's value and derivative there.
int orc_shift_knots(const double* knots, int nk, int nu, int H, double dt, int n_steps, int spline_mode,
                    double* out) {
  if (nk < 2 || nu < 1 || H < 1 || n_steps < 0 || !(dt > 0) || spline_mode < 0 || spline_mode > 2) return -1;
  const double T = H * dt, delta = T / (nk - 1);
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nu; ++j) {
      const double t = std::min(k * delta + n_steps * dt, T);
      double q, v;
      hermite_at_time<double>(knots, nk, nu, delta, t, j, &q, &v);
      out[k * nu + j] = q;
      out[(nk + k) * nu + j] = v;
    }
  // position-only variants: the shifted positions define a new spline of the same kind
  if (spline_mode != 0) position_spline_slopes<double>(spline_mode, nk, nu, delta, out);
  return 0;
}

// Knot slopes of the position-only spline variants (test access).
int orc_spline_slopes(int mode, int nk, int nu, double delta, double* knots) {
  if (nk < 2 || nu < 1 || (mode != 1 && mode != 2) || !(delta > 0)) return -1;
  position_spline_slopes<double>(mode, nk, nu, delta, knots);
  return 0;
}

int orc_sample_knots(const orc_model* m, const orc_params* p, const double* nominal, uint64_t seed,
                     uint32_t tick, int iota, int n, double* out) {
  if (!model_ok(m) || !params_ok(m, p) || iota < 0 || iota >= p->n_iters || n < 0) return -1;
  Model<double> M = load_model<double>(m);
  std::vector<double> sig(p->n_iters * p->n_knots);
  sigma_table(p, sig.data());
  sample_knots<double>(M, p, nominal, sig.data(), seed, tick, iota, n, out);
  return 0;
}

// Forward dynamics at (q, v, tau), with the soft-contact forces of that state
// when with_contacts != 0.  Optional outputs: contact forces [nc][3] (world).
int orc_forward_dynamics(const orc_model* m, const double* q, const double* v, const double* tau,
                         int with_contacts, double* qdd, double* cforce) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  Kin<double> K = kinematics(M, q, v);
  std::vector<V6<double>> fext(M.nb, V6<double>{});
  if (with_contacts) {
    ContactOut<double> C = contacts(M, K, fext);
    if (cforce)
      for (int c = 0; c < M.nc; ++c)
        for (int k = 0; k < 3; ++k) cforce[c * 3 + k] = C.force[c][k];
  }
  std::vector<double> a = aba(M, K, tau, fext);
  std::copy(a.begin(), a.end(), qdd);
  return 0;
}

// One physics step's accelerations as used inside a rollout: PD on the given
// reference (qr, vr), contact forces, and the linearly implicit terms of step
// dt.  Outputs qdd [nv], the clipped torques [n_u], the implicit joint gains
// [n_u] and the contact forces [nc][3] (world); the last three are nullable.
int orc_step_dynamics(const orc_model* m, const double* q, const double* v, const double* qr, const double* vr,
                      double dt, double* qdd, double* tau_out, double* g_out, double* cforce) {
  if (!model_ok(m) || !(dt >= 0)) return -1;
  Model<double> M = load_model<double>(m);
  PDOut<double> pd = pd_law(M, q, v, qr, vr, dt);
  Kin<double> K = kinematics(M, q, v);
  std::vector<V6<double>> fext;
  std::vector<M6<double>> Iadd;
  ContactOut<double> C = contacts(M, K, fext, dt, &Iadd);
  std::vector<double> a = aba(M, K, pd.tau.data(), fext, &Iadd, pd.g.data());
  std::copy(a.begin(), a.end(), qdd);
  if (tau_out) std::copy(pd.tau.begin(), pd.tau.end(), tau_out);
  if (g_out) std::copy(pd.g.begin(), pd.g.end(), g_out);
  if (cforce)
    for (int c = 0; c < M.nc; ++c)
      for (int k = 0; k < 3; ++k) cforce[c * 3 + k] = C.force[c][k];
  return 0;
}

// Same, in float arithmetic (diagnosis of FP32-vs-FP64 divergence only).
int orc_forward_dynamics_f32(const orc_model* m, const float* q, const float* v, const float* tau,
                             int with_contacts, float* qdd) {
  if (!model_ok(m)) return -1;
  Model<float> M = load_model<float>(m);
  Kin<float> K = kinematics(M, q, v);
  std::vector<V6<float>> fext(M.nb, V6<float>{});
  if (with_contacts) contacts(M, K, fext);
  std::vector<float> a = aba(M, K, tau, fext);
  std::copy(a.begin(), a.end(), qdd);
  return 0;
}

int orc_crba(const orc_model* m, const double* q, double* H) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  std::vector<double> v(M.nv, 0.0);
  Kin<double> K = kinematics(M, q, v.data());
  std::vector<double> Hm = crba(M, K);
  std::copy(Hm.begin(), Hm.end(), H);
  return 0;
}

int orc_rnea(const orc_model* m, const double* q, const double* v, const double* qdd, int with_contacts,
             double* tau) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  Kin<double> K = kinematics(M, q, v);
  std::vector<V6<double>> fext(M.nb, V6<double>{});
  if (with_contacts) contacts(M, K, fext);
  std::vector<double> t = rnea(M, K, qdd, fext);
  std::copy(t.begin(), t.end(), tau);
  return 0;
}

// World poses of every body: R [nb][9], p [nb][3].
int orc_body_poses(const orc_model* m, const double* q, double* R, double* p) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  std::vector<double> v(M.nv, 0.0);
  Kin<double> K = kinematics(M, q, v.data());
  for (int i = 0; i < M.nb; ++i) {
    for (int k = 0; k < 9; ++k) R[i * 9 + k] = K.Rw[i][k];
    for (int k = 0; k < 3; ++k) p[i * 3 + k] = K.pw[i][k];
  }
  return 0;
}

// The same in float arithmetic (diagnosis of FP32-vs-FP64 divergence only).
int orc_step_dynamics_f32(const orc_model* m, const float* q, const float* v, const float* qr, const float* vr,
                          float dt, float* qdd) {
  if (!model_ok(m) || !(dt >= 0)) return -1;
  Model<float> M = load_model<float>(m);
  PDOut<float> pd = pd_law(M, q, v, qr, vr, dt);
  Kin<float> K = kinematics(M, q, v);
  std::vector<V6<float>> fext;
  std::vector<M6<float>> Iadd;
  contacts(M, K, fext, dt, &Iadd);
  std::vector<float> a = aba(M, K, pd.tau.data(), fext, &Iadd, pd.g.data());
  std::copy(a.begin(), a.end(), qdd);
  return 0;
}

// One physics step of the rollout integrator from (q, v) tracking the
// reference (qr, vr): accelerations as in orc_step_dynamics, then
// v += dt qdd, q += dt v (base: position by R v_lin, quaternion by the
// exponential of the body angular velocity).  Updates q, v in place.
int orc_euler_step(const orc_model* m, double dt, double* q, double* v, const double* qr, const double* vr) {
  if (!model_ok(m) || !(dt > 0)) return -1;
  Model<double> M = load_model<double>(m);
  PDOut<double> pd = pd_law(M, q, v, qr, vr, dt);
  Kin<double> K = kinematics(M, q, v);
  std::vector<V6<double>> fext;
  std::vector<M6<double>> Iadd;
  contacts(M, K, fext, dt, &Iadd);
  std::vector<double> a = aba(M, K, pd.tau.data(), fext, &Iadd, pd.g.data());
  integrate(M, dt, q, v, a);
  return 0;
}

// Classical RK4 on (q, v) with constant torques and no contact, for the
// energy and momentum checks.  The base quaternion is advanced by its
// kinematic derivative 1/2 quat (x) (0, omega) and renormalised at the end of
// each step.
int orc_rk4(const orc_model* m, double dt, int steps, double* q, double* v, const double* tau) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  const int nq = M.nq, nv = M.nv, qo = M.fb ? 7 : 0, vo = M.fb ? 6 : 0;
  std::vector<V6<double>> fext(M.nb, V6<double>{});
  auto deriv = [&](const std::vector<double>& qq, const std::vector<double>& vv, std::vector<double>& dq,
                   std::vector<double>& dv) {
    Kin<double> K = kinematics(M, qq.data(), vv.data());
    dv = aba(M, K, tau, fext);
    dq.assign(nq, 0.0);
    for (int j = 0; j < M.nu; ++j) dq[qo + j] = vv[vo + j];
    if (M.fb) {
      M3<double> R = quat_to_R(qq.data() + 3);
      V3<double> pd = m3_v(R, V3<double>{vv[3], vv[4], vv[5]});
      for (int k = 0; k < 3; ++k) dq[k] = pd[k];
      double w = qq[3], x = qq[4], y = qq[5], z = qq[6], a = vv[0], b = vv[1], c = vv[2];
      dq[3] = 0.5 * (-x * a - y * b - z * c);
      dq[4] = 0.5 * (w * a + y * c - z * b);
      dq[5] = 0.5 * (w * b - x * c + z * a);
      dq[6] = 0.5 * (w * c + x * b - y * a);
    }
  };
  std::vector<double> Q(q, q + nq), V(v, v + nv);
  for (int s = 0; s < steps; ++s) {
    std::vector<double> k1q, k1v, k2q, k2v, k3q, k3v, k4q, k4v, tq(nq), tv(nv);
    deriv(Q, V, k1q, k1v);
    for (int k = 0; k < nq; ++k) tq[k] = Q[k] + 0.5 * dt * k1q[k];
    for (int k = 0; k < nv; ++k) tv[k] = V[k] + 0.5 * dt * k1v[k];
    deriv(tq, tv, k2q, k2v);
    for (int k = 0; k < nq; ++k) tq[k] = Q[k] + 0.5 * dt * k2q[k];
    for (int k = 0; k < nv; ++k) tv[k] = V[k] + 0.5 * dt * k2v[k];
    deriv(tq, tv, k3q, k3v);
    for (int k = 0; k < nq; ++k) tq[k] = Q[k] + dt * k3q[k];
    for (int k = 0; k < nv; ++k) tv[k] = V[k] + dt * k3v[k];
    deriv(tq, tv, k4q, k4v);
    for (int k = 0; k < nq; ++k) Q[k] += dt / 6 * (k1q[k] + 2 * k2q[k] + 2 * k3q[k] + k4q[k]);
    for (int k = 0; k < nv; ++k) V[k] += dt / 6 * (k1v[k] + 2 * k2v[k] + 2 * k3v[k] + k4v[k]);
    if (M.fb) {
      double nn = std::sqrt(Q[3] * Q[3] + Q[4] * Q[4] + Q[5] * Q[5] + Q[6] * Q[6]);
      for (int k = 3; k < 7; ++k) Q[k] /= nn;
    }
  }
  std::copy(Q.begin(), Q.end(), q);
  std::copy(V.begin(), V.end(), v);
  return 0;
}

// Mechanical energy 1/2 v^T M v - sum_i m_i g . c_i (world z up).
int orc_energy(const orc_model* m, const double* q, const double* v, double* E) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  Kin<double> K = kinematics(M, q, v);
  std::vector<double> Hm = crba(M, K);
  double T = 0;
  for (int r = 0; r < M.nv; ++r)
    for (int c = 0; c < M.nv; ++c) T += 0.5 * v[r] * Hm[r * M.nv + c] * v[c];
  double Vp = 0;
  for (int i = 0; i < M.nb; ++i) {
    V3<double> c = point_world(K, i, M.com[i]);
    Vp += M.mass[i] * M.g * c[2];
  }
  *E = T + Vp;
  return 0;
}

// Total spatial momentum expressed in world coordinates about the world origin.
int orc_momentum(const orc_model* m, const double* q, const double* v, double* h) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  Kin<double> K = kinematics(M, q, v);
  double tot[6] = {0, 0, 0, 0, 0, 0};
  for (int i = 0; i < M.nb; ++i) {
    V6<double> hb = m6_v(M.Ibody[i], K.vb[i]);
    // body -> world force transform: angular = R n + p x (R f), linear = R f
    V3<double> n = m3_v(K.Rw[i], V3<double>{hb[0], hb[1], hb[2]});
    V3<double> f = m3_v(K.Rw[i], V3<double>{hb[3], hb[4], hb[5]});
    V3<double> pf = cross(K.pw[i], f);
    for (int k = 0; k < 3; ++k) {
      tot[k] += n[k] + pf[k];
      tot[k + 3] += f[k];
    }
  }
  for (int k = 0; k < 6; ++k) h[k] = tot[k];
  return 0;
}

// Contact forces, positions, velocities and the activity mask at a state.
int orc_contacts(const orc_model* m, const double* q, const double* v, double* pos, double* vel, double* force,
                 uint32_t* mask) {
  if (!model_ok(m)) return -1;
  Model<double> M = load_model<double>(m);
  Kin<double> K = kinematics(M, q, v);
  std::vector<V6<double>> fext;
  ContactOut<double> C = contacts(M, K, fext);
  for (int c = 0; c < M.nc; ++c)
    for (int k = 0; k < 3; ++k) {
      if (pos) pos[c * 3 + k] = C.pos[c][k];
      if (vel) vel[c * 3 + k] = C.vel[c][k];
      if (force) force[c * 3 + k] = C.force[c][k];
    }
  if (mask) *mask = C.mask;
  return 0;
}

// One rollout of given sample knots from x0.  Optional debug outputs.
int orc_rollout(const orc_model* m, const orc_params* p, const double* x0, const double* knots, double* S,
                double* traj, uint32_t* masks, double* stage) {
  if (!model_ok(m) || !params_ok(m, p)) return -1;
  Model<double> M = load_model<double>(m);
  *S = rollout<double>(M, p, x0, knots, RolloutDebug<double>{traj, masks, stage});
  return 0;
}

int orc_rollout_f32(const orc_model* m, const orc_params* p, const double* x0, const double* knots, double* S,
                    uint32_t* masks) {
  if (!model_ok(m) || !params_ok(m, p)) return -1;
  Model<float> M = load_model<float>(m);
  const int nx = M.nq + M.nv, E = 2 * p->n_knots * M.nu;
  std::vector<float> x(x0, x0 + nx), th(knots, knots + E);
  *S = (double)rollout<float>(M, p, x.data(), th.data(), RolloutDebug<float>{nullptr, masks, nullptr});
  return 0;
}

// The float instantiation's trajectory (states after each control step), for
// the rounding reference of the GPU's state prediction.
int orc_rollout_f32_traj(const orc_model* m, const orc_params* p, const double* x0, const double* knots,
                         double* traj) {
  if (!model_ok(m) || !params_ok(m, p)) return -1;
  Model<float> M = load_model<float>(m);
  const int nx = M.nq + M.nv, E = 2 * p->n_knots * M.nu;
  std::vector<float> x(x0, x0 + nx), th(knots, knots + E), tr((size_t)(p->horizon + 1) * nx);
  (void)rollout<float>(M, p, x.data(), th.data(), RolloutDebug<float>{tr.data(), nullptr, nullptr});
  for (size_t i = 0; i < tr.size(); ++i) traj[i] = (double)tr[i];
  return 0;
}

}  // extern "C"

// Trajectory-forced steps (see orc_forced_steps), in T.
template <class T>
static void forced_steps(const Model<T>& M, const orc_params* p, const double* x0d, int n, const double* knots,
                         const double* traj, double* qdd, double* cost, uint32_t* masks, double* next, double* fn,
                         int threads) {
  const int H = p->horizon, nq = M.nq, nv = M.nv, nx = nq + nv, nc = M.nc, E = 2 * p->n_knots * M.nu;
  const std::vector<T> x0(x0d, x0d + nx);
#pragma omp parallel for schedule(dynamic) num_threads(threads)
  for (int r = 0; r < n; ++r) {
    const std::vector<T> th(knots + (size_t)r * E, knots + (size_t)(r + 1) * E);
    std::vector<T> q(nq), v(nv), a(nv), f(std::max(nc, 1));
    for (int h = 0; h <= H; ++h) {
      const double* xs = traj + ((size_t)r * (H + 1) + h) * nx;
      for (int k = 0; k < nq; ++k) q[k] = (T)xs[k];
      for (int k = 0; k < nv; ++k) v[k] = (T)xs[nq + k];
      if (h == H) {
        cost[(size_t)r * (H + 1) + H] = (double)terminal_cost(M, p, x0.data(), q.data(), v.data());
        break;
      }
      uint32_t mk = 0;
      const T c = control_step(M, p, th.data(), h, q.data(), v.data(), &mk, a.data(), f.data());
      const size_t rh = (size_t)r * H + h;
      cost[(size_t)r * (H + 1) + h] = (double)c;
      if (masks) masks[rh] = mk;
      if (qdd)
        for (int k = 0; k < nv; ++k) qdd[rh * nv + k] = (double)a[k];
      if (next)
        for (int k = 0; k < nx; ++k) next[rh * nx + k] = (double)(k < nq ? q[k] : v[k - nq]);
      if (fn)
        for (int k = 0; k < nc; ++k) fn[rh * nc + k] = (double)f[k];
    }
  }
}

extern "C" {

// Trajectory-forced rollout steps: for rollout r of n (knots [n][E], all from
// the initial state x0 [nq+nv]) and each control step h < H, one control step
// of the rollout from the given state traj[r][h] (traj [n][H+1][nq+nv], e.g.
// states recorded by another implementation): the accelerations of its first
// substep qdd [n][H][nv], its running cost cost[n][H+1], its contact mask
// masks [n][H], the normal force of every contact point fn [n][H][nc] and the
// state it reaches next [n][H][nq+nv]; cost[r][H] = the terminal cost at
// traj[r][H].  f32 != 0 evaluates in float.  Outputs other than cost are nullable.
int orc_forced_steps(const orc_model* m, const orc_params* p, const double* x0, int n, const double* knots,
                     const double* traj, double* qdd, double* cost, uint32_t* masks, double* next, double* fn,
                     int f32, int threads) {
  if (!model_ok(m) || !params_ok(m, p) || n < 0 || !cost) return -1;
  threads = threads < 1 ? 1 : threads;
  if (f32) {
    Model<float> M = load_model<float>(m);
    forced_steps<float>(M, p, x0, n, knots, traj, qdd, cost, masks, next, fn, threads);
  } else {
    Model<double> M = load_model<double>(m);
    forced_steps<double>(M, p, x0, n, knots, traj, qdd, cost, masks, next, fn, threads);
  }
  return 0;
}

// The integration step of a rollout alone (semi-implicit Euler with the base
// quaternion advanced by the exponential of the body angular velocity) for n
// states X [n][nq+nv] and accelerations A [n][nv], step dt: out [n][nq+nv].
int orc_integrate_batch(const orc_model* m, double dt, int n, const double* X, const double* A, double* out) {
  if (!model_ok(m) || n < 0 || !(dt >= 0)) return -1;
  Model<double> M = load_model<double>(m);
  const int nq = M.nq, nv = M.nv, nx = nq + nv;
  std::vector<double> qdd(nv);
  for (int r = 0; r < n; ++r) {
    double* q = out + (size_t)r * nx;
    std::copy(X + (size_t)r * nx, X + (size_t)(r + 1) * nx, q);
    std::copy(A + (size_t)r * nv, A + (size_t)(r + 1) * nv, qdd.begin());
    integrate(M, dt, q, q + nq, qdd);
  }
  return 0;
}

// Counts of two 3x3 matrix-vector products with the Flop scalar, y = A x,
// for the pin of the counting rules: out[0..8] for a general A, out[9..17] for
// the identity (kinds as in orc_count_ops).
int orc_count_selftest(double* out) {
  auto run = [](const double* A, double* o) {
    Flop x[3] = {0.5, -2.0, 3.0}, y[3];
    g_tally = OpTally{};
    for (int i = 0; i < 3; ++i) {
      Flop acc = 0;
      for (int j = 0; j < 3; ++j) acc += Flop(A[i * 3 + j]) * x[j];
      y[i] = acc;
    }
    (void)y;
    const OpTally& t = g_tally;
    o[0] = (double)t.add; o[1] = (double)t.mul; o[2] = (double)t.div; o[3] = (double)t.sqrt;
    o[4] = (double)t.trans; o[5] = (double)t.cmp; o[6] = (double)t.nt_add; o[7] = (double)t.nt_mul;
    o[8] = (double)t.nt_div;
  };
  const double G[9] = {1.5, 2, -3, 4, 5, 6, 7, 8, 9}, I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  run(G, out);
  run(I, out + 9);
  return 0;
}

// The arithmetic of one rollout of the Alg. 1 simulate step, counted with the
// Flop scalar (see opcount.hpp): sample n's knots drawn around `nominal` and
// clipped (iteration 0, tick 0; the Box-Muller normals themselves are formed in
// double and not counted), its H control steps from x0 and its terminal cost.
// out[0..8]: the rollout's raw add/sub, mul, div, sqrt, transcendental and
// comparison counts, then its non-trivial add/sub, mul and div counts;
// out[9..17]: the same for the sampling alone.  Model set-up is not counted.
int orc_count_ops(const orc_model* m, const orc_params* p, const double* x0, const double* nominal, uint64_t seed,
                  int n, double* out) {
  if (!model_ok(m) || !params_ok(m, p) || n < 0 || !out) return -1;
  Model<Flop> M = load_model<Flop>(m);
  const int E = 2 * p->n_knots * M.nu, nq = M.nq, nv = M.nv, H = p->horizon;
  std::vector<double> sig(p->n_iters * p->n_knots);
  sigma_table(p, sig.data());
  std::vector<Flop> nom(nominal, nominal + E), th(E), x(x0, x0 + nq + nv);
  std::vector<Flop> q(x.begin(), x.begin() + nq), v(x.begin() + nq, x.end());
  auto put = [](const OpTally& t, double* o) {
    o[0] = (double)t.add; o[1] = (double)t.mul; o[2] = (double)t.div; o[3] = (double)t.sqrt;
    o[4] = (double)t.trans; o[5] = (double)t.cmp; o[6] = (double)t.nt_add; o[7] = (double)t.nt_mul;
    o[8] = (double)t.nt_div;
  };
  g_tally = OpTally{};
  sample_knots<Flop>(M, p, nom.data(), sig.data(), seed, 0, 0, n, th.data());
  put(g_tally, out + 9);
  g_tally = OpTally{};
  sample_knots<Flop>(M, p, nom.data(), sig.data(), seed, 0, 0, n, th.data());
  for (int h = 0; h < H; ++h) (void)control_step<Flop>(M, p, th.data(), h, q.data(), v.data());
  (void)terminal_cost<Flop>(M, p, x.data(), q.data(), v.data());
  put(g_tally, out);
  return 0;
}

// Samples n0 .. n0+count-1 of iteration iota: knots generated from the
// counter-based stream and rolled out (OpenMP over samples).  Used for sampled
// parity at full problem sizes and for the CPU baseline timing.
int orc_rollouts(const orc_model* m, const orc_params* p, const double* x0, const double* nominal, uint64_t seed,
                 uint32_t tick, int iota, int n0, int count, double* S, double* samples, int threads) {
  if (!model_ok(m) || !params_ok(m, p) || iota < 0 || iota >= p->n_iters || n0 < 0 || count < 0) return -1;
  Model<double> M = load_model<double>(m);
  run_rollouts<double>(M, p, x0, nominal, seed, tick, iota, n0, count, S, samples, threads < 1 ? 1 : threads);
  return 0;
}

// Rotation angle of a unit quaternion, |log3(R)| = 2 atan2(|q_v|, |q_w|).
double orc_orientation_angle(const double* quat) { return orientation_angle<double>(quat); }

int orc_weights(int n, const double* S, double lambda, int mode, double* w, int* nstar) {
  if (n < 1 || !(lambda > 0)) return -1;
  return weights(n, S, lambda, mode, w, nstar);
}

// Weighted knot average in knot space (eq. update-nominal applied to the knots).
int orc_weighted_average(int n, int E, const double* w, const double* samples, double* out) {
  for (int e = 0; e < E; ++e) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += w[i] * samples[(size_t)i * E + e];
    out[e] = s;
  }
  return 0;
}

// The same update by the dense route: every candidate spline is evaluated at
// the node times, the dense trajectories are averaged with the weights, and
// the nominal knots are read back from the averaged position and velocity.
int orc_dense_route_update(int n, int nk, int nu, int H, double dt, const double* w, const double* samples,
                           double* out) {
  const double delta = H * dt / (nk - 1);
  const int E = 2 * nk * nu;
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nu; ++j) {
      double sq = 0, sv = 0;
      for (int i = 0; i < n; ++i) {
        double qr, vr;
        hermite_at_time<double>(samples + (size_t)i * E, nk, nu, delta, k * delta, j, &qr, &vr);
        sq += w[i] * qr;
        sv += w[i] * vr;
      }
      out[k * nu + j] = sq;
      out[nk * nu + k * nu + j] = sv;
    }
  return 0;
}

// The full MPC step (Alg. 1 inner loop): I iterations of sample -> simulate ->
// weight -> update, with best-sample tracking (Sec. III-D: strict
// improvement, lowest index among equal minima, S_best starts at +inf).
// Sampling and rollouts run in T; weights and the update in double.
}  // extern "C"
template <class T>
static int step_impl(const orc_model* m, const orc_params* p, const double* x0, const double* knots_in,
                     uint64_t seed, uint32_t tick, double* knots_out, double* best_knots, double* S_best,
                     int* best_iter, double* costs, int* n_nonfinite, int* all_nonfinite_iters, int threads) {
  Model<T> M = load_model<T>(m);
  const int N = p->n_samples, E = 2 * p->n_knots * M.nu;
  std::vector<double> nominal(knots_in, knots_in + E), S(N), w(N), samples((size_t)N * E);
  std::vector<double> best(nominal);
  double sbest = std::numeric_limits<double>::infinity();
  int bit = -1, nnf = 0, allnf = 0;
  for (int it = 0; it < p->n_iters; ++it) {
    run_rollouts<T>(M, p, x0, nominal.data(), seed, tick, it, 0, N, S.data(), samples.data(),
                    threads < 1 ? 1 : threads);
    int nstar = -1;
    int nf = weights(N, S.data(), p->lambda, p->weight_mode, w.data(), &nstar);
    nnf += N - nf;
    if (costs)
      for (int i = 0; i < N; ++i) costs[(size_t)it * N + i] = S[i];
    if (nf == 0) {
      ++allnf;
      continue;
    }
    std::vector<double> next(E);
    orc_weighted_average(N, E, w.data(), samples.data(), next.data());
    nominal = next;
    if (S[nstar] < sbest) {
      sbest = S[nstar];
      bit = it;
      std::copy(samples.begin() + (size_t)nstar * E, samples.begin() + (size_t)(nstar + 1) * E, best.begin());
    }
  }
  std::copy(nominal.begin(), nominal.end(), knots_out);
  if (best_knots) std::copy(best.begin(), best.end(), best_knots);
  if (S_best) *S_best = sbest;
  if (best_iter) *best_iter = bit;
  if (n_nonfinite) *n_nonfinite = nnf;
  if (all_nonfinite_iters) *all_nonfinite_iters = allnf;
  return 0;
}
extern "C" {

int orc_step(const orc_model* m, const orc_params* p, const double* x0, const double* knots_in, uint64_t seed,
             uint32_t tick, double* knots_out, double* best_knots, double* S_best, int* best_iter,
             double* costs, int* n_nonfinite, int* all_nonfinite_iters, int threads) {
  if (!model_ok(m) || !params_ok(m, p)) return -1;
  return step_impl<double>(m, p, x0, knots_in, seed, tick, knots_out, best_knots, S_best, best_iter, costs,
                           n_nonfinite, all_nonfinite_iters, threads);
}

// The same with sampling and rollouts in float (diagnosis of FP32 divergence only).
int orc_step_f32(const orc_model* m, const orc_params* p, const double* x0, const double* knots_in, uint64_t seed,
                 uint32_t tick, double* knots_out, double* best_knots, double* S_best, int* best_iter,
                 double* costs, int* n_nonfinite, int* all_nonfinite_iters, int threads) {
  if (!model_ok(m) || !params_ok(m, p)) return -1;
  return step_impl<float>(m, p, x0, knots_in, seed, tick, knots_out, best_knots, S_best, best_iter, costs,
                          n_nonfinite, all_nonfinite_iters, threads);
}

}  // extern "C"
