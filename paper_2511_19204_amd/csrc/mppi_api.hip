// mppi_api.hip -- host side of the C ABI in include/mppi.h: argument checks,
// model upload, per-instance device buffers, launch planning for single and
// batched steps.  Every arithmetic step of the controller runs in the kernels
// of mppi_kernels.hip; this file only validates, allocates and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <array>
#include <vector>

#include "../../include/mppi.h"
#include "mppi_dev.hpp"

namespace mppi {
// kernels (mppi_kernels.hip)
template <int G, int D, int LEG>
__global__ void rollout_kernel(const DevInst*, const int2*, int, int, const float*, const float*);
template <int G, int D, int LEG> __global__ void rollout_trace_kernel(const DevInst*, const int2*, int, int);
template <int G, int D, int LEG>
__global__ void rollout_persistent_kernel(const DevInst*, const int2*, int, unsigned int*, int, int);
template <int GC> __global__ void chain_kernel(const DevInst*, const int2*, int, int, int);
template <int G, int D> __global__ void team_kernel(const DevInst*, const int2*, int, int);
template <int G> __global__ void team_persistent_kernel(const DevInst*, const int2*, int, unsigned int*, int, int);
template <int GC> __global__ void chain_persistent_kernel(const DevInst*, const int2*, int, unsigned int*, int, int, int);
__global__ void reset_counters(unsigned int*, int);
template <int G> __global__ void sample_kernel(const DevInst*, int);
template <int G> __global__ void predict_kernel(const DevInst*, int, float*, int, int);
template <int G> __global__ void predict_batch_kernel(const PredItem*, int, int);
__global__ void shift_batch_kernel(const ShiftItem*);
__global__ void shift_knots_kernel(const float*, float*, int, int, int, int, int, float, int);
template <int G>
__global__ void dynamics_kernel(const DevModel*, int, const float*, const float*, const float*, const float*, float,
                                float*, int, int);
template <int T> __global__ void update_kernel(const DevUpdate*, const UpdateOut*, UpdateOut);
__global__ void update_single_kernel(DevUpdate);
__global__ void set_targets_kernel(DevTargets*, DevTargets);
struct StageItem {
  const float* src;
  float* dst;
  int32_t count;
};
__global__ void stage_kernel(const StageItem*);
__global__ void copy2_kernel(const float*, float*, int, const float*, float*, int);
__global__ void philox_kernel(const uint32_t*, const uint32_t*, uint32_t*, int);
}  // namespace mppi

using namespace mppi;

// A launch key selects the schedule: 0 < G <= 64 is the body schedule with G
// lanes per rollout, -GC < 0 the chain schedule with GC lanes per rollout, and
// kTeamKey + G the team schedule with G lanes per rollout.
constexpr int kTeamKey = 128;
static int key_lanes(int key) { return key > kTeamKey ? key - kTeamKey : key > 0 ? key : -key; }

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static mppi_status fail(mppi_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t _e = (expr);                                                                   \
    if (_e != hipSuccess) return fail(MPPI_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// ---------------------------------------------------------------------------
// objects
// ---------------------------------------------------------------------------
struct mppi_model {
  DevModel host;
  DevModel* dev = nullptr;
  int device = 0;
  int nq = 0, nv = 0;
};

struct mppi_ctx {
  const mppi_model* m = nullptr;
  mppi_params p{};
  uint64_t seed = 0;
  int N = 0, H = 0, K = 0, I = 0, nu = 0, E = 0, nq = 0, nv = 0, nc = 0;
  int lanes = 0;
  int device = 0;
  float delta = 0.f;
  bool regen = false;  // the update draws the samples again (samples stays unallocated)
  // device buffers
  float *sigma = nullptr, *x0 = nullptr, *nom = nullptr, *samples = nullptr, *costs = nullptr;
  float *best_state = nullptr, *f0z = nullptr, *q0 = nullptr;
  DevTargets* d_targets = nullptr;  // task targets, read by the kernels when they run
  // state prediction: measured state, trajectory knots, a cost slot, its descriptor
  float *x_meas = nullptr, *pred_knots = nullptr, *pred_cost = nullptr;
  DevInst* d_pred_inst = nullptr;
  uint32_t* tick = nullptr;
  float* upd_partial = nullptr;  // [update_shape(N).parts][E] update scratch
  uint32_t* upd_done = nullptr;  // update parts finished (0 between launches)
  DevInst* d_insts = nullptr;   // [I]
  DevUpdate* d_ups = nullptr;   // [I]
  std::vector<DevInst> h_insts;
  std::vector<DevUpdate> h_ups;
  // kernel timing (HIP events around each launch on the launch stream) when enabled
  bool profile = false;
  // per iteration: before the rollout, between rollout and update, after the update
  std::vector<std::array<hipEvent_t, 3>> ev_marks;
  std::vector<hipEvent_t> ev_pool;
};

static mppi_status ev_get(mppi_ctx* c, hipEvent_t* out) {
  if (!c->ev_pool.empty()) {
    *out = c->ev_pool.back();
    c->ev_pool.pop_back();
    return MPPI_OK;
  }
  HIP_TRY(hipEventCreate(out));
  return MPPI_OK;
}

static int next_pow2(int x) {
  int g = 4;
  while (g < x) g <<= 1;
  return g;
}

static bool valid_lanes(int G, const DevModel& M) { return (G == 4 || G == 8 || G == 16 || G == 32 || G == 64) && G >= M.nb; }


// ---------------------------------------------------------------------------
// chain schedule tables: heavy-path decomposition and the per-body rows
// ---------------------------------------------------------------------------
static void build_chain_tables(DevModel& M) {
  const int nb = M.nb;
  auto bits = [](int x) {
    float f;
    std::memcpy(&f, &x, sizeof(f));
    return f;
  };
  // subtree sizes (parents precede children) and the heavy child of every body
  std::vector<int> size(nb, 1), heavy(nb, -1);
  for (int i = nb - 1; i > 0; --i)
    if (M.parent[i] >= 0) size[M.parent[i]] += size[i];
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < M.n_child[b]; ++k) {
      const int ch = M.child[b][k];
      if (heavy[b] < 0 || size[ch] > size[heavy[b]]) heavy[b] = ch;
    }
  // chains: a body starts a chain unless it is its parent's heavy child
  std::vector<int> chain_of(nb, -1), att(nb, -1);
  int nch = 0, natt = 0;
  bool ok = M.n_levels <= kMaxLevels;
  for (int b = 0; b < nb; ++b) {
    const int lam = M.parent[b];
    if (lam >= 0 && heavy[lam] == b) continue;
    if (nch >= kMaxChains) { ok = false; break; }
    const int c = nch++;
    for (int d = 0; d < kMaxLevels; ++d) M.chain_body[c][d] = -1;
    M.chain_first[c] = M.depth[b];
    M.chain_att[c] = -1;
    if (lam >= 0) {
      if (att[lam] < 0) att[lam] = natt++;
      M.chain_att[c] = att[lam];
    }
    for (int x = b; x >= 0; x = heavy[x]) {
      chain_of[x] = c;
      if (M.depth[x] < kMaxLevels) M.chain_body[c][M.depth[x]] = x;
    }
  }
  for (int c = nch; c < kMaxChains; ++c) {
    for (int d = 0; d < kMaxLevels; ++d) M.chain_body[c][d] = -1;
    M.chain_first[c] = 0;
    M.chain_att[c] = -1;
  }
  M.chain_ok = ok ? 1 : 0;
  M.n_chains = ok ? nch : 0;
  M.n_att = natt;
  int lanes = 1;
  while (lanes < nch) lanes <<= 1;
  M.chain_lanes = lanes;
  for (int b = 0; b < nb; ++b) {
    float* r = M.rows[b];
    for (int k = 0; k < kRow; ++k) r[k] = 0.f;
    for (int k = 0; k < 27; ++k) r[row::P + k] = M.P[b][k];
    for (int k = 0; k < 3; ++k) {
      r[row::p_tree + k] = M.p_tree[b][k];
      r[row::axis_p + k] = M.axis_p[b][k];
      r[row::com + k] = M.com[b][k];
    }
    for (int k = 0; k < 6; ++k) r[row::Ic + k] = M.Ic[b][k];
    r[row::mass] = M.mass[b];
    const int j = b - M.fb;
    if (j >= 0) {
      r[row::kp] = M.kp[j]; r[row::kd] = M.kd[j]; r[row::taumax] = M.taumax[j]; r[row::arm] = M.arm[j];
    }
    r[row::parent] = bits(M.parent[b]);
    r[row::c_begin] = bits(M.c_begin[b]);
    r[row::c_count] = bits(M.c_count[b]);
    r[row::n_child] = bits(M.n_child[b]);
    r[row::heavy] = bits(heavy[b]);
    r[row::att] = bits(att[b]);
    r[row::chain] = bits(chain_of[b]);
    r[row::depth] = bits(M.depth[b]);
    for (int k = 0; k < kMaxChildren; ++k) r[row::child + k] = bits(k < M.n_child[b] ? M.child[b][k] : -1);
  }
  for (int ci = 0; ci < M.nc; ++ci) {
    for (int k = 0; k < kCt; ++k) M.ctab[ci][k] = 0.f;
    for (int k = 0; k < 3; ++k) M.ctab[ci][k] = M.cpos[ci][k];
    M.ctab[ci][4] = bits(M.corig[ci]);
  }
  // team schedule: blocks of B lanes per chain (B holds the chain's bodies and at
  // least the three coordinate lanes), a power of two of them per rollout
  int longest = 0;
  for (int c = 0; c < kMaxChains; ++c) {
    int len = 0;
    for (int d = 0; d < kMaxLevels; ++d) len += (c < M.n_chains && M.chain_body[c][d] >= 0) ? 1 : 0;
    M.chain_len[c] = len;
    longest = std::max(longest, len);
    const int first = c < M.n_chains ? M.chain_body[c][M.chain_first[c]] : -1;
    M.chain_parent[c] = first >= 0 ? M.parent[first] : -1;
  }
  int B = 4;
  while (B < longest) B <<= 1;
  int G = 1;
  while (G < M.n_chains * B) G <<= 1;
  M.team_block = B;
  M.team_lanes = G;
  M.team_ok = (M.chain_ok && M.n_chains > 0 && G <= 64) ? 1 : 0;
  // slots: bodies ranked by (depth, chain), so one level's bodies are consecutive
  M.team_slots = nb;
  for (int b = 0; b < kMaxBodies; ++b) M.team_slot[b] = 0;
  {
    std::vector<int> order(nb);
    for (int b = 0; b < nb; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return M.depth[x] != M.depth[y] ? M.depth[x] < M.depth[y] : chain_of[x] < chain_of[y];
    });
    for (int s = 0; s < nb; ++s) M.team_slot[order[s]] = s;
  }
  for (int b = 0; b < kMaxBodies; ++b)
    for (int k = 0; k < kTeamRow; ++k) M.team_rows[b][k] = 0.f;
  for (int b = 0; b < nb; ++b) {
    float* t = M.team_rows[b];
    for (int k = 0; k < 3; ++k) {
      for (int i = 0; i < 3; ++i) {
        const int col = (k + i) % 3;
        t[16 * k + i] = M.P[b][3 * k + col];
        t[16 * k + 3 + i] = M.P[b][9 + 3 * k + col];
        t[16 * k + 6 + i] = M.P[b][18 + 3 * k + col];
        t[16 * k + 9 + i] = M.p_tree[b][col];
        t[16 * k + 12 + i] = M.axis_p[b][col];
      }
    }
    const int j = b - M.fb;
    t[15] = j >= 0 ? M.arm[j] : 0.f;
    int side = 0;
    for (int c = 0; c < M.n_chains; ++c)
      if (M.chain_parent[c] == b) side |= 1 << c;
    t[16 + 15] = bits(side);
  }
}

// ---------------------------------------------------------------------------
// model
// ---------------------------------------------------------------------------
extern "C" mppi_status mppi_model_create(const mppi_model_desc* d, mppi_model** out) {
  if (!d || !out) return fail(MPPI_EINVAL, "null argument");
  const int nb = d->n_bodies;
  if (nb < 1 || nb > kMaxBodies) return fail(MPPI_EINVAL, "n_bodies must be in 1..64");
  if (d->n_contacts < 0 || d->n_contacts > kMaxContacts) return fail(MPPI_EINVAL, "n_contacts must be in 0..32");
  if (d->n_substeps < 1) return fail(MPPI_EINVAL, "n_substeps must be >= 1");
  if (!d->parent || !d->axis || !d->R_tree || !d->p_tree || !d->mass || !d->com || !d->inertia)
    return fail(MPPI_EINVAL, "null tree array");
  const int fb = d->floating_base ? 1 : 0;
  const int nu = nb - fb;
  if (nu < 1) return fail(MPPI_EINVAL, "model has no actuated joint");
  if (!d->q_min || !d->q_max || !d->tau_max || !d->kp || !d->kd) return fail(MPPI_EINVAL, "null joint array");
  if (d->n_contacts > 0 && (!d->contact_body || !d->contact_pos)) return fail(MPPI_EINVAL, "null contact array");
  if (fb && d->parent[0] != -1) return fail(MPPI_EINVAL, "floating base must be body 0 with parent -1");
  auto* m = new mppi_model();
  DevModel& M = m->host;
  std::memset(&M, 0, sizeof(M));
  M.nb = nb; M.fb = fb; M.nu = nu; M.nc = d->n_contacts; M.nsub = d->n_substeps;
  M.k = d->k_contact; M.d = d->d_contact; M.mu = d->mu; M.eps = d->eps_fric; M.g = d->gravity;
  M.ee_body = d->ee_body;
  if (d->ee_body >= nb || d->ee_body < -1) { delete m; return fail(MPPI_EINVAL, "ee_body out of range"); }
  for (int k = 0; k < 3; ++k) M.ee_pos[k] = d->ee_pos[k];
  int maxd = 0;
  for (int i = 0; i < nb; ++i) {
    const int lam = d->parent[i];
    if (lam >= i) { delete m; return fail(MPPI_EINVAL, "parent[i] must be < i"); }
    if (fb && i > 0 && lam < 0) { delete m; return fail(MPPI_EINVAL, "only the base may have parent -1"); }
    if (!(d->mass[i] > 0.f)) { delete m; return fail(MPPI_EINVAL, "masses must be positive"); }
    M.parent[i] = lam;
    M.depth[i] = lam < 0 ? (fb ? 0 : 1) : M.depth[lam] + 1;
    maxd = std::max(maxd, M.depth[i]);
    if (lam >= 0) {
      if (M.n_child[lam] >= kMaxChildren) { delete m; return fail(MPPI_EINVAL, "more than 8 children on a body"); }
      M.child[lam][M.n_child[lam]++] = i;
    }
    M.mass[i] = d->mass[i];
    M.mtot += d->mass[i];
    for (int k = 0; k < 3; ++k) { M.com[i][k] = d->com[3 * i + k]; M.p_tree[i][k] = d->p_tree[3 * i + k]; }
    for (int k = 0; k < 6; ++k) M.Ic[i][k] = d->inertia[6 * i + k];
    if (fb && i == 0) continue;
    // joint rotation C(q) = R_tree Rot(a, q) = R_tree a a^T + cos q (-R_tree K^2) + sin q (R_tree K)
    const double a[3] = {d->axis[3 * i], d->axis[3 * i + 1], d->axis[3 * i + 2]};
    const double an = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (std::fabs(an - 1.0) > 1e-4) { delete m; return fail(MPPI_EINVAL, "joint axes must be unit vectors"); }
    double Rt[9];
    for (int k = 0; k < 9; ++k) Rt[k] = d->R_tree[9 * i + k];
    const double K[9] = {0, -a[2], a[1], a[2], 0, -a[0], -a[1], a[0], 0};
    double K2[9], aa[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += K[r * 3 + k] * K[k * 3 + c];
        K2[r * 3 + c] = s;
        aa[r * 3 + c] = a[r] * a[c];
      }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double p0 = 0, p1 = 0, p2 = 0;
        for (int k = 0; k < 3; ++k) {
          p0 += Rt[r * 3 + k] * aa[k * 3 + c];
          p1 -= Rt[r * 3 + k] * K2[k * 3 + c];
          p2 += Rt[r * 3 + k] * K[k * 3 + c];
        }
        M.P[i][r * 3 + c] = (float)p0;
        M.P[i][9 + r * 3 + c] = (float)p1;
        M.P[i][18 + r * 3 + c] = (float)p2;
      }
    for (int r = 0; r < 3; ++r)
      M.axis_p[i][r] = (float)(Rt[r * 3] * a[0] + Rt[r * 3 + 1] * a[1] + Rt[r * 3 + 2] * a[2]);
    const int j = i - fb;
    M.qmin[j] = d->q_min[j]; M.qmax[j] = d->q_max[j]; M.taumax[j] = d->tau_max[j];
    M.kp[j] = d->kp[j]; M.kd[j] = d->kd[j];
    M.arm[j] = d->armature ? d->armature[j] : 0.f;
    if (!(M.arm[j] >= 0.f)) { delete m; return fail(MPPI_EINVAL, "armature must be >= 0"); }
    if (!(M.qmin[j] < M.qmax[j])) { delete m; return fail(MPPI_EINVAL, "q_min must be < q_max"); }
  }
  M.max_depth = maxd;
  M.n_levels = maxd + 1;
  // contacts grouped by body (stable within a body)
  int ci = 0;
  for (int b = 0; b < nb; ++b) {
    M.c_begin[b] = ci;
    for (int c = 0; c < d->n_contacts; ++c) {
      if (d->contact_body[c] < 0 || d->contact_body[c] >= nb) { delete m; return fail(MPPI_EINVAL, "contact_body out of range"); }
      if (d->contact_body[c] != b) continue;
      for (int k = 0; k < 3; ++k) M.cpos[ci][k] = d->contact_pos[3 * c + k];
      M.corig[ci] = c;
      ++ci;
    }
    M.c_count[b] = ci - M.c_begin[b];
  }
  build_chain_tables(M);
  m->nq = fb ? 7 + nu : nu;
  m->nv = fb ? 6 + nu : nu;
  hipError_t e1 = hipGetDevice(&m->device);
  hipError_t e2 = e1 == hipSuccess ? hipMalloc(&m->dev, sizeof(DevModel)) : e1;
  hipError_t e3 = e2 == hipSuccess ? hipMemcpy(m->dev, &M, sizeof(DevModel), hipMemcpyHostToDevice) : e2;
  if (e3 != hipSuccess) {
    if (m->dev) (void)hipFree(m->dev);
    delete m;
    return fail(MPPI_EDEVICE, std::string("model upload: ") + hipGetErrorString(e3));
  }
  *out = m;
  return MPPI_OK;
}

extern "C" mppi_status mppi_model_destroy(mppi_model* m) {
  if (!m) return fail(MPPI_EINVAL, "null model");
  if (m->dev) (void)hipFree(m->dev);
  delete m;
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
static void free_ctx_events(mppi_ctx* c) {
  for (auto& m : c->ev_marks)
    for (hipEvent_t e : m) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
}

static void free_ctx_buffers(mppi_ctx* c) {
  void* ptrs[] = {c->sigma, c->x0, c->nom, c->samples, c->costs, c->best_state, c->f0z, c->q0,
                  c->tick, c->d_insts, c->d_ups, c->x_meas, c->pred_knots, c->pred_cost, c->d_pred_inst,
                  c->upd_partial, c->upd_done, c->d_targets};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

static bool valid_target(const float* q) {
  const double n2 = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3];
  return n2 == 0.0 || std::fabs(n2 - 1.0) <= 1e-4;
}

// The device form of the task targets (an all-zero orientation target stands
// for the identity).
static DevTargets targets_of(const mppi_params& p) {
  DevTargets t{};
  t.z_des = p.z_des;
  for (int k = 0; k < 3; ++k) t.v_des[k] = p.v_des[k];
  const float* qd = p.q_des;
  const bool zero = qd[0] == 0.f && qd[1] == 0.f && qd[2] == 0.f && qd[3] == 0.f;
  const bool ident = zero || (qd[0] == 1.f && qd[1] == 0.f && qd[2] == 0.f && qd[3] == 0.f);
  t.or_target = ident ? 0 : 1;
  for (int k = 0; k < 4; ++k) t.q_des[k] = zero ? (k == 0 ? 1.f : 0.f) : qd[k];
  t.terminal_z_abs = p.terminal_z_abs ? 1 : 0;
  t.z_terminal = p.z_terminal;
  return t;
}

static void build_tables(mppi_ctx* c) {
  const DevModel& M = c->m->host;
  c->h_insts.assign(c->I, DevInst{});
  c->h_ups.assign(c->I, DevUpdate{});
  for (int it = 0; it < c->I; ++it) {
    DevInst& d = c->h_insts[it];
    d.model = c->m->dev;
    d.sigma = c->sigma;
    d.x0 = c->x0;
    d.nominal = c->nom + (size_t)(it == 0 ? 0 : 1 + (it % 2)) * c->E;
    d.samples = c->samples;
    d.costs = c->costs + (size_t)it * c->N;
    d.masks = nullptr;
    d.f0z = c->f0z;
    d.q0 = c->q0;
    d.N = c->N; d.H = c->H; d.K = c->K; d.nu = c->nu; d.E = c->E; d.iter = it; d.n_iters = c->I;
    d.cost_kind = c->p.cost_kind; d.lanes = c->lanes; d.weight_mode = c->p.weight_mode;
    d.tick_ptr = c->tick; d.tick_value = 0; d.use_tick_value = 0;
    d.seed_lo = (uint32_t)(c->seed & 0xffffffffu); d.seed_hi = (uint32_t)(c->seed >> 32);
    d.dt = c->p.dt; d.delta = c->delta; d.lambda = c->p.lambda;
    d.w_h = c->p.w_h; d.w_or = c->p.w_or; d.w_q = c->p.w_q; d.w_cv = c->p.w_cv; d.w_cf = c->p.w_cf;
    d.w_eff = c->p.w_eff; d.w_H = c->p.w_H; d.w_ee = c->p.w_ee; d.w_tau = c->p.w_tau;
    d.targets = c->d_targets;
    d.generate = 1;
    d.store_samples = c->regen ? 0 : 1;
    d.spline_mode = c->p.spline_mode;
    (void)M;
    DevUpdate& u = c->h_ups[it];
    u.costs = d.costs;
    u.samples = c->samples;
    u.regen = c->regen ? c->d_insts + it : nullptr;
    u.nominal_in = d.nominal;
    u.nominal_out = c->nom + (size_t)(1 + ((it + 1) % 2)) * c->E;
    u.weights = nullptr;
    u.best_knots = nullptr;
    u.info = nullptr;
    u.best_state = c->best_state;
    u.tick = c->tick;
    u.partial = c->upd_partial;
    u.done = c->upd_done;
    u.N = c->N; u.E = c->E; u.iter = it; u.weight_mode = c->p.weight_mode;
    u.first_iter = it == 0; u.last_iter = it == c->I - 1;
    u.parts = update_shape(c->N).parts;
    u.threads = update_shape(c->N).threads;
    u.lambda = c->p.lambda;
  }
}

extern "C" mppi_status mppi_create(const mppi_model* m, const mppi_params* p, uint64_t seed, mppi_ctx** out) {
  if (!m || !p || !out) return fail(MPPI_EINVAL, "null argument");
  if (p->n_samples < 1 || p->n_samples > 65536) return fail(MPPI_EINVAL, "n_samples must be in 1..65536");
  if (p->horizon < 1 || p->horizon > 4096) return fail(MPPI_EINVAL, "horizon must be in 1..4096");
  if (p->n_knots < 2 || p->n_knots > kMaxKnots) return fail(MPPI_EINVAL, "n_knots must be in 2..64");
  if (p->n_iters < 1 || p->n_iters > 64) return fail(MPPI_EINVAL, "n_iters must be in 1..64");
  if (!(p->dt > 0.f) || !(p->lambda > 0.f)) return fail(MPPI_EINVAL, "dt and lambda must be positive");
  if (p->weight_mode != 0 && p->weight_mode != 1) return fail(MPPI_EINVAL, "weight_mode must be 0 or 1");
  if (p->noise_mode != 0 && p->noise_mode != 1) return fail(MPPI_EINVAL, "noise_mode must be 0 or 1");
  if (p->noise_mode == 0 && !(p->beta1 > 0.f && p->beta2 > 0.f)) return fail(MPPI_EINVAL, "beta1, beta2 must be positive");
  if (p->spline_mode < 0 || p->spline_mode > 2) return fail(MPPI_EINVAL, "spline_mode must be 0, 1 or 2");
  if (!valid_target(p->q_des)) return fail(MPPI_EINVAL, "q_des must be a unit quaternion or all zero");
  const DevModel& M = m->host;
  if (p->cost_kind == 0 && M.ee_body < 0) return fail(MPPI_EINVAL, "end-effector cost needs ee_body");
  if (p->cost_kind == 1 && !M.fb) return fail(MPPI_EINVAL, "locomotion cost needs a floating base");
  if (p->cost_kind != 0 && p->cost_kind != 1) return fail(MPPI_EINVAL, "cost_kind must be 0 or 1");
  if (p->cost_kind == 1 && (!p->q0_cost || (M.nc > 0 && !p->f0z))) return fail(MPPI_EINVAL, "null q0_cost / f0z");
  if ((long)p->horizon * M.nsub * (p->n_knots - 1) >= (1L << 30)) return fail(MPPI_EINVAL, "horizon too long");
  auto* c = new mppi_ctx();
  c->m = m; c->p = *p; c->seed = seed;
  c->N = p->n_samples; c->H = p->horizon; c->K = p->n_knots; c->I = p->n_iters;
  c->nu = M.nu; c->E = 2 * c->K * c->nu; c->nq = m->nq; c->nv = m->nv; c->nc = M.nc;
  c->delta = (float)((double)p->horizon * (double)p->dt / (double)(p->n_knots - 1));
  c->lanes = next_pow2(M.nb);
  c->p.f0z = nullptr; c->p.q0_cost = nullptr;
  auto bail = [&](hipError_t e, const char* what) {
    free_ctx_buffers(c);
    delete c;
    return fail(MPPI_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipGetDevice(&c->device)) != hipSuccess) return bail(e, "hipGetDevice");
  // noise schedule in FP64, stored as float (Sec. III-B: precomputed once)
  std::vector<float> sig((size_t)c->I * c->K);
  for (int it = 0; it < c->I; ++it)
    for (int k = 0; k < c->K; ++k) {
      double s;
      if (p->noise_mode == 0)
        s = (double)p->scale_q * std::exp(-(double)it / ((double)p->beta1 * c->I) - (double)(c->K - k) / ((double)p->beta2 * c->K));
      else
        s = (double)p->sigma_lo + ((double)p->sigma_hi - (double)p->sigma_lo) * (double)k / (double)(c->K - 1);
      sig[(size_t)it * c->K + k] = (float)s;
    }
  const size_t E = c->E;
  if ((e = hipMalloc(&c->sigma, sig.size() * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc sigma");
  if ((e = hipMalloc(&c->x0, (c->nq + c->nv) * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc x0");
  if ((e = hipMalloc(&c->nom, 3 * E * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc nominal");
  // the update draws the samples' knots again from the counter-based stream when
  // they are the cubic Hermite knots in whole blocks (K n_u even); otherwise the
  // rollouts store them for it
  c->regen = (c->K * c->nu) % 2 == 0 && p->spline_mode == 0;
  if (!c->regen && (e = hipMalloc(&c->samples, (size_t)c->N * E * sizeof(float))) != hipSuccess)
    return bail(e, "hipMalloc samples");
  if ((e = hipMalloc(&c->costs, (size_t)c->I * c->N * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc costs");
  if ((e = hipMalloc(&c->best_state, (E + 5) * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc best");
  if ((e = hipMalloc(&c->f0z, std::max(M.nc, 1) * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc f0z");
  if ((e = hipMalloc(&c->q0, c->nu * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc q0");
  if ((e = hipMalloc(&c->tick, sizeof(uint32_t))) != hipSuccess) return bail(e, "hipMalloc tick");
  if ((e = hipMalloc(&c->upd_partial, (size_t)update_shape(c->N).parts * E * sizeof(float))) != hipSuccess)
    return bail(e, "hipMalloc update scratch");
  if ((e = hipMalloc(&c->upd_done, sizeof(uint32_t))) != hipSuccess) return bail(e, "hipMalloc update counter");
  if ((e = hipMalloc(&c->d_insts, c->I * sizeof(DevInst))) != hipSuccess) return bail(e, "hipMalloc insts");
  if ((e = hipMalloc(&c->d_ups, c->I * sizeof(DevUpdate))) != hipSuccess) return bail(e, "hipMalloc ups");
  if ((e = hipMalloc(&c->d_targets, sizeof(DevTargets))) != hipSuccess) return bail(e, "hipMalloc targets");
  {
    const DevTargets tg = targets_of(c->p);
    if ((e = hipMemcpy(c->d_targets, &tg, sizeof(DevTargets), hipMemcpyHostToDevice)) != hipSuccess)
      return bail(e, "upload targets");
  }
  std::vector<float> f0(std::max(M.nc, 1), 0.f), q0(c->nu, 0.f);
  if (p->f0z)
    for (int i = 0; i < M.nc; ++i) f0[i] = p->f0z[i];
  if (p->q0_cost)
    for (int i = 0; i < c->nu; ++i) q0[i] = p->q0_cost[i];
  const uint32_t zero = 0;
  if ((e = hipMemcpy(c->sigma, sig.data(), sig.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "upload sigma");
  if ((e = hipMemcpy(c->f0z, f0.data(), f0.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "upload f0z");
  if ((e = hipMemcpy(c->q0, q0.data(), q0.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "upload q0");
  if ((e = hipMemcpy(c->tick, &zero, sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "upload tick");
  if ((e = hipMemcpy(c->upd_done, &zero, sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e, "upload update counter");
  if ((e = hipMalloc(&c->x_meas, (c->nq + c->nv) * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc x_meas");
  if ((e = hipMalloc(&c->pred_knots, E * sizeof(float))) != hipSuccess) return bail(e, "hipMalloc pred knots");
  if ((e = hipMalloc(&c->pred_cost, sizeof(float))) != hipSuccess) return bail(e, "hipMalloc pred cost");
  if ((e = hipMalloc(&c->d_pred_inst, sizeof(DevInst))) != hipSuccess) return bail(e, "hipMalloc pred inst");
  build_tables(c);
  {
    // prediction: one sample, knots read (not sampled) from pred_knots, from x_meas
    DevInst d = c->h_insts[0];
    d.x0 = c->x_meas;
    d.samples = c->pred_knots;
    d.costs = c->pred_cost;
    d.masks = nullptr;
    d.N = 1;
    d.generate = 0;
    if ((e = hipMemcpy(c->d_pred_inst, &d, sizeof(DevInst), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "upload pred inst");
  }
  if ((e = hipMemcpy(c->d_insts, c->h_insts.data(), c->I * sizeof(DevInst), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "upload insts");
  if ((e = hipMemcpy(c->d_ups, c->h_ups.data(), c->I * sizeof(DevUpdate), hipMemcpyHostToDevice)) != hipSuccess) return bail(e, "upload ups");
  *out = c;
  return MPPI_OK;
}

static void purge_plans(const mppi_ctx* c);

extern "C" mppi_status mppi_destroy(mppi_ctx* c) {
  if (!c) return fail(MPPI_EINVAL, "null context");
  purge_plans(c);
  free_ctx_events(c);
  free_ctx_buffers(c);
  delete c;
  return MPPI_OK;
}

extern "C" mppi_status mppi_set_tick(mppi_ctx* c, uint32_t tick) {
  if (!c) return fail(MPPI_EINVAL, "null context");
  HIP_TRY(hipMemcpy(c->tick, &tick, sizeof(uint32_t), hipMemcpyHostToDevice));
  return MPPI_OK;
}

extern "C" mppi_status mppi_get_tick(const mppi_ctx* c, uint32_t* tick) {
  if (!c || !tick) return fail(MPPI_EINVAL, "null argument");
  HIP_TRY(hipMemcpy(tick, c->tick, sizeof(uint32_t), hipMemcpyDeviceToHost));
  return MPPI_OK;
}

extern "C" mppi_status mppi_set_targets(mppi_ctx* c, const mppi_targets* t, void* stream) {
  if (!c || !t) return fail(MPPI_EINVAL, "null argument");
  if (!valid_target(t->q_des)) return fail(MPPI_EINVAL, "q_des must be a unit quaternion or all zero");
  c->p.z_des = t->z_des;
  for (int k = 0; k < 3; ++k) c->p.v_des[k] = t->v_des[k];
  for (int k = 0; k < 4; ++k) c->p.q_des[k] = t->q_des[k];
  c->p.terminal_z_abs = t->terminal_z_abs;
  c->p.z_terminal = t->z_terminal;
  hipLaunchKernelGGL(set_targets_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, c->d_targets, targets_of(c->p));
  HIP_TRY(hipGetLastError());
  return MPPI_OK;
}

// The launch key of an instance: G > 0 selects the body schedule with G lanes per
// rollout, -GC the chain schedule with GC lanes per rollout.
static mppi_status set_key(mppi_ctx* c, int key) {
  c->lanes = key;
  for (auto& d : c->h_insts) d.lanes = key;
  HIP_TRY(hipMemcpy(c->d_insts, c->h_insts.data(), c->I * sizeof(DevInst), hipMemcpyHostToDevice));
  purge_plans(c);
  return MPPI_OK;
}

extern "C" mppi_status mppi_set_lanes_per_rollout(mppi_ctx* c, int32_t lanes) {
  if (!c) return fail(MPPI_EINVAL, "null context");
  const int G = lanes == 0 ? next_pow2(c->m->host.nb) : lanes;
  if (!valid_lanes(G, c->m->host)) return fail(MPPI_EINVAL, "lanes must be a power of two in 4..64 holding every body");
  return set_key(c, G);
}

extern "C" mppi_status mppi_get_lanes_per_rollout(const mppi_ctx* c, int32_t* lanes) {
  if (!c || !lanes) return fail(MPPI_EINVAL, "null argument");
  *lanes = key_lanes(c->lanes);
  return MPPI_OK;
}

extern "C" mppi_status mppi_set_schedule(mppi_ctx* c, int32_t schedule) {
  if (!c) return fail(MPPI_EINVAL, "null context");
  const DevModel& M = c->m->host;
  if (schedule == MPPI_SCHEDULE_BODY) return set_key(c, next_pow2(M.nb));
  if (schedule == MPPI_SCHEDULE_TEAM) {
    if (!M.team_ok) return fail(MPPI_EINVAL, "tree has more than 8 chains, depth above 15 or needs more than 64 lanes");
    return set_key(c, kTeamKey + M.team_lanes);
  }
  if (schedule != MPPI_SCHEDULE_CHAIN) return fail(MPPI_EINVAL, "unknown schedule");
  if (!M.chain_ok) return fail(MPPI_EINVAL, "tree has more than 8 chains or depth above 15");
  return set_key(c, -M.chain_lanes);
}

extern "C" mppi_status mppi_get_schedule(const mppi_ctx* c, int32_t* schedule) {
  if (!c || !schedule) return fail(MPPI_EINVAL, "null argument");
  *schedule = c->lanes > kTeamKey ? MPPI_SCHEDULE_TEAM : c->lanes > 0 ? MPPI_SCHEDULE_BODY : MPPI_SCHEDULE_CHAIN;
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------


// Largest per-instance sizes of one launch (they size the LDS regions).
// A legged tree: a floating base with serial chains hanging off it, numbered
// depth first (every joint body's parent is the previous body, or the base for
// a chain's first body, and no body but the base has more than one child).
static bool legged(const DevModel& M) {
  if (!M.fb || M.nb < 2) return false;
  for (int b = 1; b < M.nb; ++b) {
    if (M.parent[b] != b - 1 && M.parent[b] != 0) return false;
    if (M.n_child[b] > 1) return false;
  }
  return true;
}
// A legged tree of four chains of three bodies (the quadruped's shape) with at
// most one contact point per body.
static bool legged_4x3(const DevModel& M) {
  if (!legged(M) || M.nb != 13) return false;
  for (int b = 0; b < M.nb; ++b)
    if (M.c_count[b] > 1) return false;
  for (int k = 0; k < 4; ++k)
    if (M.parent[1 + 3 * k] != 0 || M.parent[2 + 3 * k] != 1 + 3 * k || M.parent[3 + 3 * k] != 2 + 3 * k) return false;
  return true;
}

// A fixed-base serial chain: body b's parent is body b - 1, the first body's the
// world.
static bool serial_chain(const DevModel& M) {
  if (M.fb || M.nb < 1 || M.parent[0] != -1) return false;
  for (int b = 1; b < M.nb; ++b)
    if (M.parent[b] != b - 1) return false;
  return true;
}

struct Dims {
  int E = 0, nb = 0, nc = 0, nch = 0, natt = 0, ns = 0, depth = 0;
  // every instance added is a legged tree / of four chains of three / a serial chain
  bool leg = true, quad = true, serial = true;
  void add(const mppi_ctx* c) {
    const DevModel& M = c->m->host;
    leg = leg && legged(M);
    quad = quad && legged_4x3(M);
    serial = serial && serial_chain(M);
    E = std::max(E, c->E);
    nb = std::max(nb, M.nb);
    nc = std::max(nc, M.nc);
    nch = std::max(nch, M.n_chains);
    natt = std::max(natt, M.n_att);
    ns = std::max(ns, M.team_slots);
    depth = std::max(depth, M.max_depth);
  }
};
static Dims dims_of(const mppi_ctx* c) {
  Dims d;
  d.add(c);
  return d;
}

// LDS a chain-schedule block may take: two blocks per compute unit (160 KiB).
constexpr int kChainLdsBudget = 64 * 1024;

struct LaunchShape {
  int stride = 0, table = 0, lds = 0, groups = 0;  // groups = rollouts per block
};
static LaunchShape launch_shape(int key, const Dims& dm) {
  LaunchShape sh;
  if (key > kTeamKey) {
    const int G = key - kTeamKey;
    sh.stride = team_layout(G, dm.ns, dm.E, dm.nch).total;
    sh.table = team_table_floats(dm.ns, dm.nc);
    sh.groups = 64 / G;
    sh.lds = (sh.table + sh.groups * sh.stride) * (int)sizeof(float);
  } else if (key > 0) {
    sh.stride = group_floats(key, dm.E);
    sh.table = body_sched_table_floats(dm.nb, dm.nc);
    sh.groups = 64 / key;
    sh.lds = (sh.table + sh.groups * sh.stride) * (int)sizeof(float);
  } else {
    const int GC = -key;
    sh.stride = chain_group_floats(GC, dm.nb, dm.E, dm.nch, dm.natt);
    sh.table = chain_table_floats(dm.nb, dm.nc);
    const int fit = (kChainLdsBudget / (int)sizeof(float) - sh.table) / sh.stride;
    sh.groups = std::max(1, std::min(64 / GC, fit));
    sh.lds = (sh.table + sh.groups * sh.stride) * (int)sizeof(float);
  }
  return sh;
}
static int rollouts_per_block(int key, const Dims& dm) { return launch_shape(key, dm).groups; }

// the body schedule's kernel for trees at most 3 or 6 levels deep has its level
// loops unrolled; deeper trees take the general one
template <int G>
static hipError_t launch_rollout_G(int blocks, const DevInst* insts, const int2* work, const LaunchShape& sh,
                                   const Dims& dm, hipStream_t s, const float* x0_in, const float* nominal_in) {
  const int depth = dm.depth;
  if constexpr (G == 16) {
    if (depth <= 3 && dm.quad) {
      hipLaunchKernelGGL((rollout_kernel<16, 3, 2>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride,
                         sh.table, x0_in, nominal_in);
      return hipGetLastError();
    }
  }
  if constexpr (G >= 8 && G <= 32) {
    if (depth <= 3 && dm.leg) {
      hipLaunchKernelGGL((rollout_kernel<G, 3, 1>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride,
                         sh.table, x0_in, nominal_in);
      return hipGetLastError();
    }
  }
  if constexpr (G == 4 || G == 8) {
    if (depth <= 3 && dm.serial) {
      hipLaunchKernelGGL((rollout_kernel<G, 3, 3>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride,
                         sh.table, x0_in, nominal_in);
      return hipGetLastError();
    }
  }
  if (depth <= 3)
    hipLaunchKernelGGL((rollout_kernel<G, 3, 0>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride, sh.table,
                       x0_in, nominal_in);
  else if (depth <= 6)
    hipLaunchKernelGGL((rollout_kernel<G, 6, 0>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride, sh.table,
                       x0_in, nominal_in);
  else
    hipLaunchKernelGGL((rollout_kernel<G, 0, 0>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride, sh.table,
                       x0_in, nominal_in);
  return hipGetLastError();
}
template <int G>
static hipError_t launch_team_G(int blocks, const DevInst* insts, const int2* work, const LaunchShape& sh, int depth,
                                hipStream_t s) {
  if (depth <= 3)
    hipLaunchKernelGGL((team_kernel<G, 3>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride, sh.table);
  else if (depth <= 6)
    hipLaunchKernelGGL((team_kernel<G, 6>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride, sh.table);
  else
    hipLaunchKernelGGL((team_kernel<G, 0>), dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride, sh.table);
  return hipGetLastError();
}
template <int GC>
static hipError_t launch_chain_GC(int blocks, const DevInst* insts, const int2* work, const LaunchShape& sh,
                                  hipStream_t s) {
  hipLaunchKernelGGL(chain_kernel<GC>, dim3(blocks), dim3(64), sh.lds, s, insts, work, sh.stride, sh.table, sh.groups);
  return hipGetLastError();
}

// x0_in / nominal_in (body schedule, one instance; else null): state and nominal to
// use instead of the instance's staged copies.
static hipError_t launch_rollout(int key, int blocks, const DevInst* insts, const int2* work, const Dims& dm,
                                 hipStream_t s, const float* x0_in = nullptr, const float* nominal_in = nullptr) {
  if ((x0_in || nominal_in) && !(key > 0 && key < kTeamKey)) return hipErrorInvalidValue;
  const LaunchShape sh = launch_shape(key, dm);
  switch (key) {
    case 4: return launch_rollout_G<4>(blocks, insts, work, sh, dm, s, x0_in, nominal_in);
    case 8: return launch_rollout_G<8>(blocks, insts, work, sh, dm, s, x0_in, nominal_in);
    case 16: return launch_rollout_G<16>(blocks, insts, work, sh, dm, s, x0_in, nominal_in);
    case 32: return launch_rollout_G<32>(blocks, insts, work, sh, dm, s, x0_in, nominal_in);
    case 64: return launch_rollout_G<64>(blocks, insts, work, sh, dm, s, x0_in, nominal_in);
    case kTeamKey + 4: return launch_team_G<4>(blocks, insts, work, sh, dm.depth, s);
    case kTeamKey + 8: return launch_team_G<8>(blocks, insts, work, sh, dm.depth, s);
    case kTeamKey + 16: return launch_team_G<16>(blocks, insts, work, sh, dm.depth, s);
    case kTeamKey + 32: return launch_team_G<32>(blocks, insts, work, sh, dm.depth, s);
    case kTeamKey + 64: return launch_team_G<64>(blocks, insts, work, sh, dm.depth, s);
    case -1: return launch_chain_GC<1>(blocks, insts, work, sh, s);
    case -2: return launch_chain_GC<2>(blocks, insts, work, sh, s);
    case -4: return launch_chain_GC<4>(blocks, insts, work, sh, s);
    case -8: return launch_chain_GC<8>(blocks, insts, work, sh, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename Kern, typename... Args>
static hipError_t launch_persistent_k(Kern kern, int n_items, const LaunchShape& sh, unsigned int* counter,
                                      hipStream_t s, Args... args) {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, sh.lds);
  const int grid = std::min(n_items, std::max(1, cus) * std::max(1, per_cu));
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, counter, 1);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(64), sh.lds, s, args...);
  return hipGetLastError();
}

// the persistent body-schedule kernel with the specialisation launch_rollout_G would take
template <int G>
static hipError_t launch_persistent_body(int n_items, const LaunchShape& sh, const Dims& dm, unsigned int* counter,
                                         hipStream_t s, const DevInst* insts, const int2* work) {
#define P_ARGS n_items, sh, counter, s, insts, work, n_items, counter, sh.stride, sh.table
  if constexpr (G == 16)
    if (dm.depth <= 3 && dm.quad) return launch_persistent_k(rollout_persistent_kernel<16, 3, 2>, P_ARGS);
  if constexpr (G >= 8 && G <= 32)
    if (dm.depth <= 3 && dm.leg) return launch_persistent_k(rollout_persistent_kernel<G, 3, 1>, P_ARGS);
  if constexpr (G == 4 || G == 8)
    if (dm.depth <= 3 && dm.serial) return launch_persistent_k(rollout_persistent_kernel<G, 3, 3>, P_ARGS);
  if (dm.depth <= 3) return launch_persistent_k(rollout_persistent_kernel<G, 3, 0>, P_ARGS);
  if (dm.depth <= 6) return launch_persistent_k(rollout_persistent_kernel<G, 6, 0>, P_ARGS);
  return launch_persistent_k(rollout_persistent_kernel<G, 0, 0>, P_ARGS);
#undef P_ARGS
}

static hipError_t launch_persistent(int key, int n_items, const DevInst* insts, const int2* work, const Dims& dm,
                                    unsigned int* counter, hipStream_t s) {
  const LaunchShape sh = launch_shape(key, dm);
#define BODY_P(G) launch_persistent_body<G>(n_items, sh, dm, counter, s, insts, work)
#define CHAIN_P(GC) launch_persistent_k(chain_persistent_kernel<GC>, n_items, sh, counter, s, insts, work, n_items, counter, sh.stride, sh.table, sh.groups)
#define TEAM_P(G) launch_persistent_k(team_persistent_kernel<G>, n_items, sh, counter, s, insts, work, n_items, counter, sh.stride, sh.table)
  switch (key) {
    case 4: return BODY_P(4);
    case 8: return BODY_P(8);
    case 16: return BODY_P(16);
    case 32: return BODY_P(32);
    case 64: return BODY_P(64);
    case kTeamKey + 4: return TEAM_P(4);
    case kTeamKey + 8: return TEAM_P(8);
    case kTeamKey + 16: return TEAM_P(16);
    case kTeamKey + 32: return TEAM_P(32);
    case kTeamKey + 64: return TEAM_P(64);
    case -1: return CHAIN_P(1);
    case -2: return CHAIN_P(2);
    case -4: return CHAIN_P(4);
    case -8: return CHAIN_P(8);
    default: return hipErrorInvalidValue;
  }
#undef BODY_P
#undef CHAIN_P
#undef TEAM_P
}

static std::atomic<int> g_persistent{0};

// Grid of an iteration's update launches over a table of instances ordered with
// the 64-thread updates first (update_shape): n64 instances of at most parts64
// parts, then n256 of at most parts256.
struct UpdGrid {
  int n64 = 0, parts64 = 1, n256 = 0, parts256 = 1;
  void add(const DevUpdate& u) {
    if (u.threads == 64) {
      ++n64;
      parts64 = std::max(parts64, u.parts);
    } else {
      ++n256;
      parts256 = std::max(parts256, u.parts);
    }
  }
};
// instance order for such a table: the 64-thread updates first, otherwise as given
static void order_by_update_shape(std::vector<int>& idx, const std::function<int(int)>& n_of) {
  std::stable_partition(idx.begin(), idx.end(), [&](int i) { return update_shape(n_of(i)).threads == 64; });
}
static hipError_t launch_updates(const DevUpdate* ups, const UpdateOut* outs, const UpdGrid& g, hipStream_t s) {
  const UpdateOut none{nullptr, nullptr, nullptr, nullptr};
  if (g.n64 > 0) hipLaunchKernelGGL(update_kernel<64>, dim3(g.parts64, g.n64), dim3(64), 0, s, ups, outs, none);
  if (g.n256 > 0)
    hipLaunchKernelGGL(update_kernel<kUpdThreads>, dim3(g.parts256, g.n256), dim3(kUpdThreads), 0, s, ups + g.n64,
                       outs ? outs + g.n64 : nullptr, none);
  return hipGetLastError();
}
// one instance's update (its shape), with the call's outputs o
static hipError_t launch_update1(const DevUpdate* u, const DevUpdate& h, const UpdateOut& o, hipStream_t s) {
  if (h.threads == 64) hipLaunchKernelGGL(update_kernel<64>, dim3(h.parts, 1), dim3(64), 0, s, u, nullptr, o);
  else hipLaunchKernelGGL(update_kernel<kUpdThreads>, dim3(h.parts, 1), dim3(kUpdThreads), 0, s, u, nullptr, o);
  return hipGetLastError();
}

extern "C" mppi_status mppi_set_batch_options(const mppi_batch_opts* o) {
  if (!o) return fail(MPPI_EINVAL, "null options");
  g_persistent = o->persistent ? 1 : 0;
  return MPPI_OK;
}

// The I planning iterations of one step from the staged state (c->x0) and
// nominal (c->nom), as a sequence of rollout and update launches on s.
// x0_in / nominal_in (nullable, body schedule only): the call's state and initial
// nominal read in place, instead of staged copies.
static mppi_status run_iterations(mppi_ctx* c, float* d_knots_out, float* d_best_knots, mppi_step_info* d_info,
                                  float* d_costs, hipStream_t s, const float* x0_in = nullptr,
                                  const float* nominal_in = nullptr) {
  const Dims dm = dims_of(c);
  const int R = rollouts_per_block(c->lanes, dm);
  const int blocks = (c->N + R - 1) / R;
  for (int it = 0; it < c->I; ++it) {
    // timing marks: the rollout runs between marks 0 and 1, the update between 1 and 2
    std::array<hipEvent_t, 3> mk{};
    if (c->profile) {
      for (hipEvent_t& e : mk) {
        mppi_status st = ev_get(c, &e);
        if (st != MPPI_OK) return st;
      }
      HIP_TRY(hipEventRecord(mk[0], s));
    }
    const float* nom0 = it == 0 ? nominal_in : nullptr;
    HIP_TRY(launch_rollout(c->lanes, blocks, c->d_insts + it, nullptr, dm, s, x0_in, nom0));
    if (c->profile) HIP_TRY(hipEventRecord(mk[1], s));
    UpdateOut o{nullptr, nullptr, nullptr, nom0};
    if (it == c->I - 1) o = UpdateOut{d_knots_out, d_best_knots, d_info, nom0};
    HIP_TRY(launch_update1(c->d_ups + it, c->h_ups[it], o, s));
    if (c->profile) {
      HIP_TRY(hipEventRecord(mk[2], s));
      c->ev_marks.push_back(mk);
    }
  }
  if (d_costs) HIP_TRY(hipMemcpyAsync(d_costs, c->costs, (size_t)c->I * c->N * sizeof(float), hipMemcpyDeviceToDevice, s));
  return MPPI_OK;
}

extern "C" mppi_status mppi_step(mppi_ctx* c, const float* d_state, const float* d_knots_in, float* d_knots_out,
                                 float* d_best_knots, mppi_step_info* d_info, float* d_costs, void* stream) {
  if (!c || !d_state || !d_knots_in || !d_knots_out) return fail(MPPI_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  // the body schedule reads the state and the warm-start knots in place; the
  // others take copies in the instance's buffers (one launch)
  if (c->lanes > 0 && c->lanes < kTeamKey)
    return run_iterations(c, d_knots_out, d_best_knots, d_info, d_costs, s, d_state, d_knots_in);
  hipLaunchKernelGGL(copy2_kernel, dim3(2), dim3(64), 0, s, d_state, c->x0, c->nq + c->nv, d_knots_in, c->nom, c->E);
  HIP_TRY(hipGetLastError());
  return run_iterations(c, d_knots_out, d_best_knots, d_info, d_costs, s);
}

// ---------------------------------------------------------------------------
// state prediction and warm start (Sec. III-E)
// ---------------------------------------------------------------------------
template <int G>
static hipError_t launch_predict_G(const mppi_ctx* c, int steps, float* out, hipStream_t s) {
  const int table = body_sched_table_floats(c->m->host.nb, c->nc);
  const int stride = group_floats(G, c->E);
  const int lds = (table + (64 / G) * stride) * (int)sizeof(float);
  hipLaunchKernelGGL(predict_kernel<G>, dim3(1), dim3(64), lds, s, c->d_pred_inst, steps, out, stride, table);
  return hipGetLastError();
}

// state_out <- state reached from c->x_meas along c->pred_knots after `steps` control steps
static mppi_status launch_predict(const mppi_ctx* c, int steps, float* out, hipStream_t s) {
  hipError_t e;
  switch (next_pow2(c->m->host.nb)) {
    case 4: e = launch_predict_G<4>(c, steps, out, s); break;
    case 8: e = launch_predict_G<8>(c, steps, out, s); break;
    case 16: e = launch_predict_G<16>(c, steps, out, s); break;
    case 32: e = launch_predict_G<32>(c, steps, out, s); break;
    default: e = launch_predict_G<64>(c, steps, out, s); break;
  }
  HIP_TRY(e);
  return MPPI_OK;
}

static mppi_status launch_shift(const mppi_ctx* c, const float* in, int steps, float* out, hipStream_t s) {
  hipLaunchKernelGGL(shift_knots_kernel, dim3(1), dim3(kShiftThreads), 0, s, in, out, c->K, c->nu, c->H * c->m->host.nsub,
                     c->m->host.nsub, std::min(steps, c->H), c->delta, c->p.spline_mode);
  HIP_TRY(hipGetLastError());
  return MPPI_OK;
}

extern "C" mppi_status mppi_predict(mppi_ctx* c, const float* d_state_in, const float* d_knots, int32_t n_steps,
                                    float* d_state_out, void* stream) {
  if (!c || !d_state_in || !d_knots || !d_state_out) return fail(MPPI_EINVAL, "null argument");
  if (n_steps < 0 || n_steps > c->H) return fail(MPPI_EINVAL, "n_steps must be in 0..horizon");
  hipStream_t s = (hipStream_t)stream;
  const size_t nx = (size_t)(c->nq + c->nv) * sizeof(float);
  HIP_TRY(hipMemcpyAsync(c->x_meas, d_state_in, nx, hipMemcpyDeviceToDevice, s));
  if (n_steps == 0) {
    HIP_TRY(hipMemcpyAsync(d_state_out, c->x_meas, nx, hipMemcpyDeviceToDevice, s));
    return MPPI_OK;
  }
  HIP_TRY(hipMemcpyAsync(c->pred_knots, d_knots, c->E * sizeof(float), hipMemcpyDeviceToDevice, s));
  return launch_predict(c, n_steps, d_state_out, s);
}

extern "C" mppi_status mppi_shift_knots(mppi_ctx* c, const float* d_knots_in, int32_t n_steps, float* d_knots_out,
                                        void* stream) {
  if (!c || !d_knots_in || !d_knots_out) return fail(MPPI_EINVAL, "null argument");
  if (n_steps < 0) return fail(MPPI_EINVAL, "n_steps must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(c->pred_knots, d_knots_in, c->E * sizeof(float), hipMemcpyDeviceToDevice, s));
  return launch_shift(c, c->pred_knots, n_steps, d_knots_out, s);
}

// The part of a tick before the iterations: the instance's x0 becomes the
// measured state carried n_delay control steps along tau_best, and its nominal
// becomes tau_best shifted by n_delay actions.
static mppi_status tick_prefix(mppi_ctx* c, const float* d_state_meas, int32_t n_delay, const float* d_best,
                               float* d_state_pred, hipStream_t s) {
  const size_t nx = (size_t)(c->nq + c->nv) * sizeof(float);
  // x_t: the measured state carried n_delay control steps along tau_best
  hipLaunchKernelGGL(copy2_kernel, dim3(2), dim3(64), 0, s, d_state_meas, c->x_meas, c->nq + c->nv, d_best,
                     c->pred_knots, c->E);
  HIP_TRY(hipGetLastError());
  if (n_delay == 0) {
    HIP_TRY(hipMemcpyAsync(c->x0, c->x_meas, nx, hipMemcpyDeviceToDevice, s));
  } else {
    mppi_status st = launch_predict(c, n_delay, c->x0, s);
    if (st != MPPI_OK) return st;
  }
  if (d_state_pred) HIP_TRY(hipMemcpyAsync(d_state_pred, c->x0, nx, hipMemcpyDeviceToDevice, s));
  // tau_0 <- tau_best shifted by n_delay actions (final action repeated)
  return launch_shift(c, c->pred_knots, n_delay, c->nom, s);
}

extern "C" mppi_status mppi_tick(mppi_ctx* c, const float* d_state_meas, int32_t n_delay, float* d_best,
                                 float* d_knots_out, mppi_step_info* d_info, float* d_state_pred, void* stream) {
  if (!c || !d_state_meas || !d_best) return fail(MPPI_EINVAL, "null argument");
  if (n_delay < 0 || n_delay > c->H) return fail(MPPI_EINVAL, "n_delay must be in 0..horizon");
  hipStream_t s = (hipStream_t)stream;
  mppi_status st = tick_prefix(c, d_state_meas, n_delay, d_best, d_state_pred, s);
  if (st != MPPI_OK) return st;
  // I iterations; the best simulated trajectory replaces tau_best
  float* nominal_out = d_knots_out ? d_knots_out : c->pred_knots;  // consumed by the shift already
  return run_iterations(c, nominal_out, d_best, d_info, nullptr, s);
}

// ---------------------------------------------------------------------------
// batched steps: cached launch plans keyed by the instance list
// ---------------------------------------------------------------------------
namespace {
struct GroupLaunch {
  int G = 0, blocks = 0;
  Dims dims;
  int2* work = nullptr;            // device [blocks]
  unsigned int* counter = nullptr; // device work counter of the persistent form
};
struct IterPlan {
  DevInst* insts = nullptr;     // device, indexed by work.x
  DevUpdate* ups = nullptr;     // device [n_active]
  std::vector<int> active;      // instance indices (into the batch) active in this iteration
  std::vector<GroupLaunch> groups;
  UpdGrid upd;                  // update launches (active holds the 64-thread updates first)
};
struct Plan {
  std::vector<const mppi_ctx*> ctxs;
  int device = 0;
  std::vector<IterPlan> iters;
  ~Plan() {
    (void)hipDeviceSynchronize();  // kernels of earlier calls may still read these tables
    for (auto& it : iters) {
      if (it.insts) (void)hipFree(it.insts);
      if (it.ups) (void)hipFree(it.ups);
      for (auto& g : it.groups) {
        if (g.work) (void)hipFree(g.work);
        if (g.counter) (void)hipFree(g.counter);
      }
    }
  }
};
// per-call argument block in a pool of pinned host buffers that the kernels read
// in place
struct RingSlot {
  void* host = nullptr;
  void* dev = nullptr;  // the same memory's device address
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
std::mutex g_mu;
std::vector<std::unique_ptr<Plan>> g_plans;
// launch-table buffers of batched launches (a deque: entries never move)
std::deque<RingSlot> g_ring;
}  // namespace

static void purge_plans(const mppi_ctx* c) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans.erase(std::remove_if(g_plans.begin(), g_plans.end(),
                               [&](const std::unique_ptr<Plan>& p) {
                                 return std::find(p->ctxs.begin(), p->ctxs.end(), c) != p->ctxs.end();
                               }),
                g_plans.end());
}

static mppi_status build_plan(const std::vector<const mppi_ctx*>& ctxs, Plan** out) {
  auto plan = std::make_unique<Plan>();
  plan->ctxs = ctxs;
  HIP_TRY(hipGetDevice(&plan->device));
  int Imax = 0;
  for (auto* c : ctxs) Imax = std::max(Imax, c->I);
  plan->iters.resize(Imax);
  for (int it = 0; it < Imax; ++it) {
    IterPlan& ip = plan->iters[it];
    std::vector<DevInst> hi;
    std::vector<DevUpdate> hu;
    for (int i = 0; i < (int)ctxs.size(); ++i)
      if (ctxs[i]->I > it) ip.active.push_back(i);
    order_by_update_shape(ip.active, [&](int i) { return ctxs[i]->N; });
    for (int i : ip.active) {
      hi.push_back(ctxs[i]->h_insts[it]);
      hu.push_back(ctxs[i]->h_ups[it]);
      ip.upd.add(hu.back());
    }
    HIP_TRY(hipMalloc(&ip.insts, hi.size() * sizeof(DevInst)));
    HIP_TRY(hipMemcpy(ip.insts, hi.data(), hi.size() * sizeof(DevInst), hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&ip.ups, hu.size() * sizeof(DevUpdate)));
    HIP_TRY(hipMemcpy(ip.ups, hu.data(), hu.size() * sizeof(DevUpdate), hipMemcpyHostToDevice));
    // one launch per lane count; inside it the longest rollouts first
    std::map<int, std::vector<int>> byG;
    for (int a = 0; a < (int)ip.active.size(); ++a) byG[ctxs[ip.active[a]]->lanes].push_back(a);
    for (auto& kv : byG) {
      GroupLaunch gl;
      gl.G = kv.first;
      for (int a : kv.second) gl.dims.add(ctxs[ip.active[a]]);
      const int R = rollouts_per_block(gl.G, gl.dims);
      std::vector<int> order = kv.second;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const mppi_ctx* cx = ctxs[ip.active[x]];
        const mppi_ctx* cy = ctxs[ip.active[y]];
        return (long)cx->H * cx->m->host.nsub * cx->m->host.nb > (long)cy->H * cy->m->host.nsub * cy->m->host.nb;
      });
      std::vector<int2> work;
      for (int a : order) {
        const mppi_ctx* c = ctxs[ip.active[a]];
        for (int n0 = 0; n0 < c->N; n0 += R) work.push_back(make_int2(a, n0));
      }
      gl.blocks = (int)work.size();
      HIP_TRY(hipMalloc(&gl.counter, sizeof(unsigned int)));
      HIP_TRY(hipMalloc(&gl.work, work.size() * sizeof(int2)));
      HIP_TRY(hipMemcpy(gl.work, work.data(), work.size() * sizeof(int2), hipMemcpyHostToDevice));
      ip.groups.push_back(gl);
    }
  }
  *out = plan.get();
  g_plans.push_back(std::move(plan));
  if (g_plans.size() > 32) g_plans.erase(g_plans.begin());
  return MPPI_OK;
}

// A launch-table buffer that no kernel reads any more: the first entry whose
// last reader has finished (its event, recorded after that kernel on whichever
// stream ran it, has completed), or a new entry when every one is still in use.
// Never waits: a batch on one stream must not stall behind another stream's
// longer work (the pool grows to the number of batches in flight at once).
static mppi_status ring_slot(size_t bytes, RingSlot** out) {
  RingSlot* found = nullptr;
  for (RingSlot& e : g_ring) {
    if (e.pending) {
      const hipError_t q = hipEventQuery(e.ev);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return fail(MPPI_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(q));
      e.pending = false;
    }
    found = &e;
    break;
  }
  if (!found) {
    g_ring.emplace_back();
    found = &g_ring.back();
  }
  RingSlot& r = *found;
  if (r.cap < bytes) {
    if (r.host) (void)hipHostFree(r.host);
    r.host = r.dev = nullptr;
    size_t cap = std::max<size_t>(bytes, 4096);
    // pinned host memory that the kernels read in place (no upload copy: a copy
    // is a blit kernel, which on a device full of rollouts waits for a free slot)
    HIP_TRY(hipHostMalloc(&r.host, cap));
    HIP_TRY(hipHostGetDevicePointer(&r.dev, r.host, 0));
    r.cap = cap;
  }
  if (!r.ev) HIP_TRY(hipEventCreateWithFlags(&r.ev, hipEventDisableTiming));
  *out = &r;
  return MPPI_OK;
}

extern "C" mppi_status mppi_step_batch(int32_t n, mppi_ctx* const* ctxs, const float* const* d_states,
                                       const float* const* d_knots_in, float* const* d_knots_out,
                                       float* const* d_best_knots, mppi_step_info* const* d_infos, void* stream) {
  if (n < 1 || !ctxs || !d_states || !d_knots_in || !d_knots_out) return fail(MPPI_EINVAL, "null argument");
  std::vector<const mppi_ctx*> list(n);
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !d_states[i] || !d_knots_in[i] || !d_knots_out[i]) return fail(MPPI_EINVAL, "null entry");
    list[i] = ctxs[i];
    for (int k = 0; k < i; ++k)
      if (list[k] == list[i]) return fail(MPPI_EINVAL, "an instance appears twice in one batch");
  }
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(g_mu);
  Plan* plan = nullptr;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  for (auto& p : g_plans)
    if (p->ctxs == list && p->device == dev) { plan = p.get(); break; }
  if (!plan) {
    mppi_status st = build_plan(list, &plan);
    if (st != MPPI_OK) return st;
  }
  // per-call block: stage items [2n], then per-iteration output tables
  const int Imax = (int)plan->iters.size();
  size_t n_out = 0;
  for (auto& ip : plan->iters) n_out += ip.active.size();
  const size_t bytes = 2 * n * sizeof(StageItem) + n_out * sizeof(UpdateOut);
  RingSlot* r = nullptr;
  mppi_status st = ring_slot(bytes, &r);
  if (st != MPPI_OK) return st;
  auto* items = reinterpret_cast<StageItem*>(r->host);
  for (int i = 0; i < n; ++i) {
    items[2 * i] = StageItem{d_states[i], list[i]->x0, list[i]->nq + list[i]->nv};
    items[2 * i + 1] = StageItem{d_knots_in[i], list[i]->nom, list[i]->E};
  }
  auto* outs = reinterpret_cast<UpdateOut*>(items + 2 * n);
  std::vector<size_t> out_off(Imax);
  size_t off = 0;
  for (int it = 0; it < Imax; ++it) {
    out_off[it] = off;
    for (int a : plan->iters[it].active) {
      const bool last = list[a]->I - 1 == it;
      outs[off++] = last ? UpdateOut{d_knots_out[a], d_best_knots ? d_best_knots[a] : nullptr,
                                     d_infos ? (void*)d_infos[a] : nullptr}
                         : UpdateOut{nullptr, nullptr, nullptr};
    }
  }
  // the slot is reusable only once every kernel reading its tables has finished:
  // its event is recorded after the last of them (below), since another call may
  // run on another stream
  r->pending = true;
  auto* d_items = reinterpret_cast<StageItem*>(r->dev);
  auto* d_outs = reinterpret_cast<UpdateOut*>(d_items + 2 * n);
  hipLaunchKernelGGL(stage_kernel, dim3(2 * n), dim3(64), 0, s, d_items);
  HIP_TRY(hipGetLastError());
  for (int it = 0; it < Imax; ++it) {
    IterPlan& ip = plan->iters[it];
    for (auto& g : ip.groups) {
      if (g_persistent)
        HIP_TRY(launch_persistent(g.G, g.blocks, ip.insts, g.work, g.dims, g.counter, s));
      else
        HIP_TRY(launch_rollout(g.G, g.blocks, ip.insts, g.work, g.dims, s));
    }
    HIP_TRY(launch_updates(ip.ups, d_outs + out_off[it], ip.upd, s));
  }
  HIP_TRY(hipEventRecord(r->ev, s));
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// graphs: a fixed batch captured once (tables uploaded at creation; the graph
// holds kernels only) and replayed; every replay is one MPC step of every
// instance and advances their ticks
// ---------------------------------------------------------------------------
struct mppi_graph {
  Plan* plan = nullptr;
  std::vector<const mppi_ctx*> ctxs;
  void* dev_block = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" mppi_status mppi_graph_create(int32_t n, mppi_ctx* const* ctxs, const float* const* d_states,
                                         const float* const* d_knots_in, float* const* d_knots_out,
                                         float* const* d_best_knots, mppi_step_info* const* d_infos,
                                         mppi_graph** out) {
  if (n < 1 || !ctxs || !d_states || !d_knots_in || !d_knots_out || !out) return fail(MPPI_EINVAL, "null argument");
  std::vector<const mppi_ctx*> list(n);
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !d_states[i] || !d_knots_in[i] || !d_knots_out[i]) return fail(MPPI_EINVAL, "null entry");
    list[i] = ctxs[i];
    for (int k = 0; k < i; ++k)
      if (list[k] == list[i]) return fail(MPPI_EINVAL, "an instance appears twice in one batch");
  }
  std::lock_guard<std::mutex> lk(g_mu);
  // a graph owns its own plan (not the shared cache, which may evict)
  Plan* plan = nullptr;
  mppi_status st = build_plan(list, &plan);
  if (st != MPPI_OK) return st;
  auto owned = std::move(g_plans.back());
  g_plans.pop_back();
  const int Imax = (int)plan->iters.size();
  size_t n_out = 0;
  for (auto& ip : plan->iters) n_out += ip.active.size();
  const size_t bytes = 2 * n * sizeof(StageItem) + n_out * sizeof(UpdateOut);
  std::vector<char> host(bytes);
  auto* items = reinterpret_cast<StageItem*>(host.data());
  for (int i = 0; i < n; ++i) {
    items[2 * i] = StageItem{d_states[i], list[i]->x0, list[i]->nq + list[i]->nv};
    items[2 * i + 1] = StageItem{d_knots_in[i], list[i]->nom, list[i]->E};
  }
  auto* outs = reinterpret_cast<UpdateOut*>(items + 2 * n);
  std::vector<size_t> out_off(Imax);
  size_t off = 0;
  for (int it = 0; it < Imax; ++it) {
    out_off[it] = off;
    for (int a : plan->iters[it].active) {
      const bool last = list[a]->I - 1 == it;
      outs[off++] = last ? UpdateOut{d_knots_out[a], d_best_knots ? d_best_knots[a] : nullptr,
                                     d_infos ? (void*)d_infos[a] : nullptr}
                         : UpdateOut{nullptr, nullptr, nullptr};
    }
  }
  auto g = std::make_unique<mppi_graph>();
  HIP_TRY(hipMalloc(&g->dev_block, bytes));
  HIP_TRY(hipMemcpy(g->dev_block, host.data(), bytes, hipMemcpyHostToDevice));
  auto* d_items = reinterpret_cast<StageItem*>(g->dev_block);
  auto* d_outs = reinterpret_cast<UpdateOut*>(d_items + 2 * n);
  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(stage_kernel, dim3(2 * n), dim3(64), 0, cs, d_items);
    for (int it = 0; it < Imax && e == hipSuccess; ++it) {
      IterPlan& ip = plan->iters[it];
      for (auto& gl : ip.groups) {
        e = g_persistent ? launch_persistent(gl.G, gl.blocks, ip.insts, gl.work, gl.dims, gl.counter, cs)
                         : launch_rollout(gl.G, gl.blocks, ip.insts, gl.work, gl.dims, cs);
        if (e != hipSuccess) break;
      }
      if (e == hipSuccess) e = launch_updates(ip.ups, d_outs + out_off[it], ip.upd, cs);
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e == hipSuccess) e = e2;
    g->graph = graph;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipFree(g->dev_block);
    return fail(MPPI_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  g->plan = owned.release();
  g->ctxs = list;
  *out = g.release();
  return MPPI_OK;
}

extern "C" mppi_status mppi_graph_launch(mppi_graph* g, void* stream) {
  if (!g || !g->exec) return fail(MPPI_EINVAL, "null graph");
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return MPPI_OK;
}

extern "C" mppi_status mppi_graph_destroy(mppi_graph* g) {
  if (!g) return fail(MPPI_EINVAL, "null graph");
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->dev_block) (void)hipFree(g->dev_block);
  delete g->plan;
  delete g;
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// autotuner: lanes per rollout of one instance, by timing real steps
// ---------------------------------------------------------------------------
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<const mppi_model*, int, int, int>, int> g_tuned;
}

extern "C" mppi_status mppi_autotune(mppi_ctx* c, const float* d_state, const float* d_knots, int32_t reps,
                                     void* stream, int32_t* best_lanes) {
  if (!c || !d_state || !d_knots) return fail(MPPI_EINVAL, "null argument");
  const auto key = std::make_tuple(c->m, c->N, c->H, c->K);
  auto report = [&](int k) {
    if (best_lanes) *best_lanes = k > 0 ? k : -k;
  };
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      mppi_status st = set_key(c, it->second);
      if (st == MPPI_OK) report(it->second);
      return st;
    }
  }
  // candidates: the body schedule at every lane count that holds the tree, and the chain schedule
  const DevModel& M = c->m->host;
  std::vector<int> cand;
  for (int G = next_pow2(M.nb); G <= 64; G *= 2) cand.push_back(G);
  if (M.chain_ok) cand.push_back(-M.chain_lanes);
  if (M.team_ok) cand.push_back(kTeamKey + M.team_lanes);
  hipStream_t s = (hipStream_t)stream;
  uint32_t tick0 = 0;
  HIP_TRY(hipMemcpy(&tick0, c->tick, sizeof(uint32_t), hipMemcpyDeviceToHost));
  float* scratch = nullptr;
  HIP_TRY(hipMalloc(&scratch, c->E * sizeof(float)));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = c->lanes;
  float best_ms = 1e30f;
  reps = std::max(1, reps);
  for (int k : cand) {
    mppi_status st = set_key(c, k);
    if (st != MPPI_OK) break;
    st = mppi_step(c, d_state, d_knots, scratch, nullptr, nullptr, nullptr, s);  // warm-up
    if (st != MPPI_OK) break;
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) {
      st = mppi_step(c, d_state, d_knots, scratch, nullptr, nullptr, nullptr, s);
      if (st != MPPI_OK) break;
    }
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) { best_ms = ms; best = k; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(scratch);
  HIP_TRY(hipMemcpy(c->tick, &tick0, sizeof(uint32_t), hipMemcpyHostToDevice));
  mppi_status st = set_key(c, best);
  if (st != MPPI_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
  }
  report(best);
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// verification entry points
// ---------------------------------------------------------------------------
extern "C" mppi_status mppi_debug_philox(const uint32_t* d_ctr, const uint32_t* d_key, uint32_t* d_out, int32_t n,
                                         void* stream) {
  if (n < 0 || (n > 0 && (!d_ctr || !d_key || !d_out))) return fail(MPPI_EINVAL, "bad arguments");
  if (n == 0) return MPPI_OK;
  hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_ctr, d_key, d_out, n);
  HIP_TRY(hipGetLastError());
  return MPPI_OK;
}

template <int G>
static hipError_t launch_samples_G(const DevInst* inst, int N, int E, hipStream_t s) {
  const int R = 64 / G;
  const int lds = (kTabContacts + R * group_floats(G, E)) * (int)sizeof(float);
  hipLaunchKernelGGL(sample_kernel<G>, dim3((N + R - 1) / R), dim3(64), lds, s, inst, group_floats(G, E));
  return hipGetLastError();
}

// A scratch DevInst (device) for verification launches, released after the stream drains.
static mppi_status debug_inst(const DevInst& h, hipStream_t s, DevInst** out) {
  DevInst* d = nullptr;
  HIP_TRY(hipMalloc(&d, sizeof(DevInst)));
  HIP_TRY(hipMemcpyAsync(d, &h, sizeof(DevInst), hipMemcpyHostToDevice, s));
  *out = d;
  return MPPI_OK;
}

extern "C" mppi_status mppi_debug_samples(mppi_ctx* c, const float* d_knots_in, int32_t iter, uint32_t tick,
                                          float* d_samples, void* stream) {
  if (!c || !d_knots_in || !d_samples || iter < 0 || iter >= c->I) return fail(MPPI_EINVAL, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  DevInst h = c->h_insts[iter];
  h.nominal = d_knots_in;
  h.samples = d_samples;
  h.store_samples = 1;
  h.use_tick_value = 1;
  h.tick_value = tick;
  DevInst* d = nullptr;
  mppi_status st = debug_inst(h, s, &d);
  if (st != MPPI_OK) return st;
  hipError_t e;
  switch (c->lanes > 0 && c->lanes <= 64 ? c->lanes : next_pow2(c->m->host.nb)) {
    case 4: e = launch_samples_G<4>(d, c->N, c->E, s); break;
    case 8: e = launch_samples_G<8>(d, c->N, c->E, s); break;
    case 16: e = launch_samples_G<16>(d, c->N, c->E, s); break;
    case 32: e = launch_samples_G<32>(d, c->N, c->E, s); break;
    default: e = launch_samples_G<64>(d, c->N, c->E, s); break;
  }
  HIP_TRY(e);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipFree(d));
  return MPPI_OK;
}

template <int G>
static hipError_t launch_dyn_G(const mppi_model* m, int n, const float* q, const float* v, const float* qr,
                               const float* vr, float dt, float* qdd, hipStream_t s) {
  const int R = 64 / G;
  const int table = body_sched_table_floats(m->host.nb, m->host.nc);
  const int lds = (table + R * group_floats(G, 0)) * (int)sizeof(float);
  hipLaunchKernelGGL(dynamics_kernel<G>, dim3((n + R - 1) / R), dim3(64), lds, s, m->dev, n, q, v, qr, vr, dt, qdd,
                     group_floats(G, 0), table);
  return hipGetLastError();
}

extern "C" mppi_status mppi_debug_dynamics(const mppi_model* m, int32_t n, const float* d_q, const float* d_v,
                                           const float* d_qref, const float* d_vref, float dt, float* d_qdd,
                                           void* stream) {
  if (!m || n < 0 || !(dt >= 0.f)) return fail(MPPI_EINVAL, "bad arguments");
  if (n == 0) return MPPI_OK;
  if (!d_q || !d_v || !d_qref || !d_vref || !d_qdd) return fail(MPPI_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const int G = next_pow2(m->host.nb);
  hipError_t e;
  switch (G) {
    case 4: e = launch_dyn_G<4>(m, n, d_q, d_v, d_qref, d_vref, dt, d_qdd, s); break;
    case 8: e = launch_dyn_G<8>(m, n, d_q, d_v, d_qref, d_vref, dt, d_qdd, s); break;
    case 16: e = launch_dyn_G<16>(m, n, d_q, d_v, d_qref, d_vref, dt, d_qdd, s); break;
    case 32: e = launch_dyn_G<32>(m, n, d_q, d_v, d_qref, d_vref, dt, d_qdd, s); break;
    default: e = launch_dyn_G<64>(m, n, d_q, d_v, d_qref, d_vref, dt, d_qdd, s); break;
  }
  HIP_TRY(e);
  return MPPI_OK;
}

extern "C" mppi_status mppi_debug_rollouts(mppi_ctx* c, const float* d_state, const float* d_samples, float* d_costs,
                                           uint32_t* d_masks, void* stream) {
  if (!c || !d_state || !d_samples || !d_costs) return fail(MPPI_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  DevInst h = c->h_insts[0];
  h.x0 = d_state;
  h.samples = const_cast<float*>(d_samples);
  h.costs = d_costs;
  h.masks = d_masks;
  h.generate = 0;
  DevInst* d = nullptr;
  mppi_status st = debug_inst(h, s, &d);
  if (st != MPPI_OK) return st;
  const int R = rollouts_per_block(c->lanes, dims_of(c));
  HIP_TRY(launch_rollout(c->lanes, (c->N + R - 1) / R, d, nullptr, dims_of(c), s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipFree(d));
  return MPPI_OK;
}

// The traced twin of launch_rollout for one instance of the body schedule: the
// same grid, block, LDS layout and depth specialisation as mppi_step's launch.
template <int G>
static hipError_t launch_trace_G(const DevInst* inst, int N, const LaunchShape& sh, const Dims& dm, hipStream_t s) {
  const int blocks = (N + sh.groups - 1) / sh.groups;
  const int depth = dm.depth;
  if constexpr (G == 16) {
    if (depth <= 3 && dm.quad) {
      hipLaunchKernelGGL((rollout_trace_kernel<16, 3, 2>), dim3(blocks), dim3(64), sh.lds, s, inst, nullptr,
                         sh.stride, sh.table);
      return hipGetLastError();
    }
  }
  if constexpr (G >= 8 && G <= 32) {
    if (depth <= 3 && dm.leg) {
      hipLaunchKernelGGL((rollout_trace_kernel<G, 3, 1>), dim3(blocks), dim3(64), sh.lds, s, inst, nullptr,
                         sh.stride, sh.table);
      return hipGetLastError();
    }
  }
  if constexpr (G == 4 || G == 8) {
    if (depth <= 3 && dm.serial) {
      hipLaunchKernelGGL((rollout_trace_kernel<G, 3, 3>), dim3(blocks), dim3(64), sh.lds, s, inst, nullptr,
                         sh.stride, sh.table);
      return hipGetLastError();
    }
  }
  if (depth <= 3)
    hipLaunchKernelGGL((rollout_trace_kernel<G, 3, 0>), dim3(blocks), dim3(64), sh.lds, s, inst, nullptr, sh.stride, sh.table);
  else if (depth <= 6)
    hipLaunchKernelGGL((rollout_trace_kernel<G, 6, 0>), dim3(blocks), dim3(64), sh.lds, s, inst, nullptr, sh.stride, sh.table);
  else
    hipLaunchKernelGGL((rollout_trace_kernel<G, 0, 0>), dim3(blocks), dim3(64), sh.lds, s, inst, nullptr, sh.stride, sh.table);
  return hipGetLastError();
}
static hipError_t launch_trace(int key, const DevInst* inst, int N, const Dims& dm, hipStream_t s) {
  const LaunchShape sh = launch_shape(key, dm);
  switch (key) {
    case 4: return launch_trace_G<4>(inst, N, sh, dm, s);
    case 8: return launch_trace_G<8>(inst, N, sh, dm, s);
    case 16: return launch_trace_G<16>(inst, N, sh, dm, s);
    case 32: return launch_trace_G<32>(inst, N, sh, dm, s);
    case 64: return launch_trace_G<64>(inst, N, sh, dm, s);
    default: return hipErrorInvalidValue;
  }
}

extern "C" mppi_status mppi_debug_trace(mppi_ctx* c, const float* d_state, const float* d_knots_in, int32_t iter,
                                        uint32_t tick, const int32_t* d_trace_map, float* d_trace, float* d_samples,
                                        float* d_costs, uint32_t* d_masks, void* stream) {
  if (!c || !d_state || !d_knots_in || !d_trace_map || !d_trace || !d_samples || !d_costs || !d_masks)
    return fail(MPPI_EINVAL, "null argument");
  if (iter < 0 || iter >= c->I) return fail(MPPI_EINVAL, "iter must be in 0..n_iters-1");
  if (!(c->lanes > 0 && c->lanes < kTeamKey)) return fail(MPPI_EINVAL, "tracing needs the body schedule");
  hipStream_t s = (hipStream_t)stream;
  DevInst h = c->h_insts[iter];
  h.x0 = d_state;
  h.nominal = d_knots_in;
  h.samples = d_samples;
  h.store_samples = 1;
  h.costs = d_costs;
  h.masks = d_masks;
  h.use_tick_value = 1;
  h.tick_value = tick;
  h.trace = d_trace;
  h.trace_map = d_trace_map;
  DevInst* d = nullptr;
  mppi_status st = debug_inst(h, s, &d);
  if (st != MPPI_OK) return st;
  HIP_TRY(launch_trace(c->lanes, d, c->N, dims_of(c), s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipFree(d));
  return MPPI_OK;
}

extern "C" mppi_status mppi_debug_update(mppi_ctx* c, const float* d_costs, const float* d_samples,
                                         const float* d_knots_in, float* d_knots_out, float* d_weights, void* stream) {
  if (!c || !d_costs || !d_samples || !d_knots_in || !d_knots_out) return fail(MPPI_EINVAL, "null argument");
  hipStream_t s = (hipStream_t)stream;
  DevUpdate h = c->h_ups[0];
  h.costs = d_costs;
  h.samples = d_samples;
  h.regen = nullptr;  // the same parts as the context's own update, so the same sums
  h.nominal_in = d_knots_in;
  h.nominal_out = d_knots_out;
  h.weights = d_weights;
  h.first_iter = 1;
  h.last_iter = 0;
  h.tick = nullptr;
  DevUpdate* d = nullptr;
  HIP_TRY(hipMalloc(&d, sizeof(DevUpdate)));
  HIP_TRY(hipMemcpyAsync(d, &h, sizeof(DevUpdate), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_update1(d, h, UpdateOut{nullptr, nullptr, nullptr, nullptr}, s));
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipFree(d));
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// the update without allocation: its scratch in a fixed device array
// ---------------------------------------------------------------------------
// Layout (floats): [kNaParts][kNaMaxE] per-slice weighted sums, then the
// running-best record [kNaMaxE + 5], then the finished-slice counter (as bits).
constexpr int kNaMaxE = 8192;
constexpr int kNaMaxN = 65536;
constexpr size_t kNaPartial = (size_t)kUpdMaxParts * kNaMaxE;
constexpr size_t kNaBest = kNaPartial;
constexpr size_t kNaCounter = kNaBest + kNaMaxE + 8;
constexpr size_t kNaFloats = kNaCounter + 64;
static __device__ __align__(256) float scratch[kNaFloats];

// The scratch's device address per device (the array's host-side name is not a
// device address), looked up once per device with that device current.
static std::mutex g_na_mu;
static std::unordered_map<int, float*> g_na_ptr;

static mppi_status noalloc_scratch(float** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_na_mu);
  auto it = g_na_ptr.find(dev);
  if (it != g_na_ptr.end()) {
    *out = it->second;
    return MPPI_OK;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(MPPI_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_na_ptr[dev] = static_cast<float*>(ptr);
  *out = static_cast<float*>(ptr);
  return MPPI_OK;
}

extern "C" mppi_status mppi_update_noalloc(int32_t n_samples, int32_t n_elems, float lambda, int32_t weight_mode,
                                           const float* d_costs, const float* d_samples, const float* d_knots_in,
                                           float* d_knots_out, float* d_weights, void* stream) {
  if (!d_costs || !d_samples || !d_knots_in || !d_knots_out) return fail(MPPI_EINVAL, "null argument");
  if (n_samples < 1 || n_samples > kNaMaxN) return fail(MPPI_EINVAL, "n_samples must be in 1..65536");
  if (n_elems < 1 || n_elems > kNaMaxE) return fail(MPPI_EINVAL, "n_elems must be in 1..8192");
  if (!(lambda > 0.f)) return fail(MPPI_EINVAL, "lambda must be positive");
  if (weight_mode != 0 && weight_mode != 1) return fail(MPPI_EINVAL, "weight_mode must be 0 or 1");
  if ((n_elems & 3) == 0 && (reinterpret_cast<uintptr_t>(d_samples) & 15) != 0)
    return fail(MPPI_EINVAL, "d_samples must be 16-byte aligned when n_elems is a multiple of 4");
  float* base = nullptr;
  mppi_status st = noalloc_scratch(&base);
  if (st != MPPI_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  DevUpdate u{};
  u.costs = d_costs;
  u.samples = d_samples;
  u.nominal_in = d_knots_in;
  u.nominal_out = d_knots_out;
  u.weights = d_weights;
  u.best_state = base + kNaBest;
  u.partial = base;
  u.done = reinterpret_cast<uint32_t*>(base + kNaCounter);
  u.N = n_samples;
  u.E = n_elems;
  u.weight_mode = weight_mode;
  u.first_iter = 1;
  u.parts = update_parts(n_samples);
  u.threads = kUpdThreads;
  u.lambda = lambda;
  // the counter is left at zero by every complete launch; cleared here too (a
  // fill kernel, so the call can be captured in a graph) in case an earlier
  // launch on this device never finished
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, u.done, 1);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(update_single_kernel, dim3(u.parts), dim3(kUpdThreads), 0, s, u);
  HIP_TRY(hipGetLastError());
  return MPPI_OK;
}

extern "C" const char* mppi_last_error(void) { return g_err.c_str(); }
extern "C" const char* mppi_version(void) { return "mppi-gfx950 0.1"; }

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
extern "C" mppi_status mppi_profile_enable(mppi_ctx* c, int32_t on) {
  if (!c) return fail(MPPI_EINVAL, "null context");
  c->profile = on != 0;
  return MPPI_OK;
}

extern "C" mppi_status mppi_profile_read(mppi_ctx* c, double* rollout_ms, int32_t* n_rollout, double* update_ms,
                                         int32_t* n_update) {
  if (!c || !rollout_ms || !n_rollout || !update_ms || !n_update) return fail(MPPI_EINVAL, "null argument");
  double tr = 0, tu = 0;
  for (auto& m : c->ev_marks) {
    HIP_TRY(hipEventSynchronize(m[2]));
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, m[0], m[1]));
    HIP_TRY(hipEventElapsedTime(&b, m[1], m[2]));
    tr += a;
    tu += b;
  }
  *rollout_ms = tr;
  *n_rollout = (int32_t)c->ev_marks.size();
  *update_ms = tu;
  *n_update = (int32_t)c->ev_marks.size();
  for (auto& m : c->ev_marks)
    for (hipEvent_t e : m) c->ev_pool.push_back(e);
  c->ev_marks.clear();
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// batches of arbitrary composition without device allocation: launch tables
// built on the host in a pinned buffer of the pool, which the kernels read in place
// ---------------------------------------------------------------------------
struct BatchReq {
  mppi_ctx* ctx;
  const float* state;     // a step: its state; a tick: the measured state
  const float* knots_in;  // a step: its warm-start nominal (a tick starts from best_out)
  float* knots_out;       // outputs of the last iteration (each nullable)
  float* best_out = nullptr;        // a tick's tau_best (in/out)
  mppi_step_info* info_out = nullptr;
  int32_t n_delay = 0;              // a tick's prediction steps
  bool tick = false;                // prediction and warm-start shift before the iterations
  // the slice of the request's iterations this launch runs: it0 .. it0+n_it-1
  // (n_it < 0: to the last).  The staging copies and a tick's prefix run with
  // iteration 0; the outputs are written by the last iteration.
  int32_t it0 = 0;
  int32_t n_it = -1;
};

// Prediction groups of a batch's ticks by lane count: the launch shape covers the
// largest instance of the group.
static int pred_lanes(const mppi_ctx* c) {
  const int g = next_pow2(c->m->host.nb);
  return g < 4 ? 4 : (g > 64 ? 64 : g);
}
static hipError_t launch_predict_batch(int G, int n_items, const PredItem* items, int stride, int table,
                                       hipStream_t s) {
  const int lds = (table + (64 / G) * stride) * (int)sizeof(float);
  switch (G) {
    case 4: hipLaunchKernelGGL(predict_batch_kernel<4>, dim3(n_items), dim3(64), lds, s, items, stride, table); break;
    case 8: hipLaunchKernelGGL(predict_batch_kernel<8>, dim3(n_items), dim3(64), lds, s, items, stride, table); break;
    case 16: hipLaunchKernelGGL(predict_batch_kernel<16>, dim3(n_items), dim3(64), lds, s, items, stride, table); break;
    case 32: hipLaunchKernelGGL(predict_batch_kernel<32>, dim3(n_items), dim3(64), lds, s, items, stride, table); break;
    default: hipLaunchKernelGGL(predict_batch_kernel<64>, dim3(n_items), dim3(64), lds, s, items, stride, table); break;
  }
  return hipGetLastError();
}

// Streams onto which an iteration's rollout groups fork: group 0 runs on the
// launch stream, group k on aux[(k-1) % n_aux] after ev_fork recorded on the
// launch stream; the launch stream waits for ev_join[j] recorded on aux[j] before
// the iteration's update.  Groups of different lane counts then run side by side
// instead of one after the other.
struct ForkStreams {
  const hipStream_t* aux = nullptr;
  int n_aux = 0;
  hipEvent_t ev_fork = nullptr;
  const hipEvent_t* ev_join = nullptr;
};

static mppi_status launch_batch_dynamic(const std::vector<BatchReq>& reqs, unsigned int* counters, int n_counters,
                                        bool persistent, hipStream_t s, const ForkStreams* fork = nullptr) {
  const int n = (int)reqs.size();
  // iterations of request i in this launch: it0(i) .. it0(i)+n_iters[i]-1
  std::vector<int> n_iters(n);
  int Imax = 0;
  for (int i = 0; i < n; ++i) {
    const int left = reqs[i].ctx->I - reqs[i].it0;
    if (reqs[i].it0 < 0 || left < 1) return fail(MPPI_EINVAL, "iteration slice outside the instance's iterations");
    n_iters[i] = reqs[i].n_it < 0 ? left : std::min(reqs[i].n_it, left);
    Imax = std::max(Imax, n_iters[i]);
  }
  struct GroupDesc { int G; Dims dims; size_t work_off; int n_items; };
  // upd: the update launches' grids (the active list holds the 64-thread
  // updates first); blocks beyond an instance's own parts return at once but
  // would still wait for a free slot on a busy device
  struct IterDesc { size_t inst_off, up_off, out_off; int n_active; UpdGrid upd; std::vector<GroupDesc> groups; };
  std::vector<IterDesc> iters(Imax);
  // requests starting at iteration 0 stage their inputs; ticks among them run
  // their prefixes (prediction by lane count, then the shifts) after the staging
  // copies and before the iterations
  std::vector<int> staged, ticks;
  std::map<int, std::vector<int>> pred_groups;
  for (int i = 0; i < n; ++i) {
    if (reqs[i].it0 != 0) continue;
    staged.push_back(i);
    if (reqs[i].tick) {
      ticks.push_back(i);
      pred_groups[pred_lanes(reqs[i].ctx)].push_back(i);
    }
  }
  const int ns = (int)staged.size(), nt = (int)ticks.size();
  // sizes
  size_t bytes = 2 * ns * sizeof(StageItem);
  std::vector<std::vector<int>> active(Imax);
  for (int it = 0; it < Imax; ++it) {
    for (int i = 0; i < n; ++i)
      if (n_iters[i] > it) active[it].push_back(i);
    order_by_update_shape(active[it], [&](int i) { return reqs[i].ctx->N; });
  }
  auto align = [](size_t x) { return (x + 255) & ~size_t(255); };
  bytes = align(bytes);
  const size_t pred_off = bytes;
  bytes = align(bytes + nt * sizeof(PredItem));
  const size_t shift_off = bytes;
  bytes = align(bytes + nt * sizeof(ShiftItem));
  for (int it = 0; it < Imax; ++it) {
    IterDesc& d = iters[it];
    d.n_active = (int)active[it].size();
    d.inst_off = bytes; bytes = align(bytes + d.n_active * sizeof(DevInst));
    d.up_off = bytes; bytes = align(bytes + d.n_active * sizeof(DevUpdate));
    d.out_off = bytes; bytes = align(bytes + d.n_active * sizeof(UpdateOut));
    std::map<int, std::vector<int>> byG;
    for (int a = 0; a < d.n_active; ++a) byG[reqs[active[it][a]].ctx->lanes].push_back(a);
    for (auto& kv : byG) {
      GroupDesc g{kv.first, Dims{}, bytes, 0};
      for (int a : kv.second) g.dims.add(reqs[active[it][a]].ctx);
      const int R = rollouts_per_block(g.G, g.dims);
      for (int a : kv.second) g.n_items += (reqs[active[it][a]].ctx->N + R - 1) / R;
      bytes = align(bytes + g.n_items * sizeof(int2));
      d.groups.push_back(g);
    }
  }
  RingSlot* r = nullptr;
  mppi_status st = ring_slot(bytes, &r);
  if (st != MPPI_OK) return st;
  char* h = reinterpret_cast<char*>(r->host);
  char* dv = reinterpret_cast<char*>(r->dev);
  auto* items = reinterpret_cast<StageItem*>(h);
  for (int k = 0; k < ns; ++k) {
    const BatchReq& q = reqs[staged[k]];
    mppi_ctx* c = q.ctx;
    if (q.tick) {  // measured state and tau_best into the prediction buffers
      items[2 * k] = StageItem{q.state, c->x_meas, c->nq + c->nv};
      items[2 * k + 1] = StageItem{q.best_out, c->pred_knots, c->E};
    } else {
      items[2 * k] = StageItem{q.state, c->x0, c->nq + c->nv};
      items[2 * k + 1] = StageItem{q.knots_in, c->nom, c->E};
    }
  }
  {
    // predictions grouped by lane count (consecutive in the table), then the shifts
    auto* hp = reinterpret_cast<PredItem*>(h + pred_off);
    int k = 0;
    for (auto& kv : pred_groups)
      for (int i : kv.second) hp[k++] = PredItem{reqs[i].ctx->d_pred_inst, reqs[i].ctx->x0, reqs[i].n_delay};
    auto* hs = reinterpret_cast<ShiftItem*>(h + shift_off);
    for (int t = 0; t < nt; ++t) {
      const mppi_ctx* c = reqs[ticks[t]].ctx;
      hs[t] = ShiftItem{c->pred_knots, c->nom, c->K, c->nu, c->H * c->m->host.nsub, c->m->host.nsub,
                        std::min(reqs[ticks[t]].n_delay, c->H), c->p.spline_mode, c->delta};
    }
  }
  for (int it = 0; it < Imax; ++it) {
    IterDesc& d = iters[it];
    auto* hi = reinterpret_cast<DevInst*>(h + d.inst_off);
    auto* hu = reinterpret_cast<DevUpdate*>(h + d.up_off);
    auto* ho = reinterpret_cast<UpdateOut*>(h + d.out_off);
    for (int a = 0; a < d.n_active; ++a) {
      const BatchReq& q = reqs[active[it][a]];
      const int ci = q.it0 + it;  // the instance's own iteration index
      hi[a] = q.ctx->h_insts[ci];
      // served rounds: trees deeper than three levels (the longest per-step
      // chains, on the critical path of their rounds) issue first where their
      // wavefronts share a SIMD with others
      hi[a].wave_prio = q.ctx->m->host.max_depth > 3 ? 3 : 0;
      hu[a] = q.ctx->h_ups[ci];
      d.upd.add(hu[a]);
      ho[a] = q.ctx->I - 1 == ci ? UpdateOut{q.knots_out, q.best_out, q.info_out} : UpdateOut{nullptr, nullptr, nullptr};
    }
    std::map<int, std::vector<int>> byG;
    for (int a = 0; a < d.n_active; ++a) byG[reqs[active[it][a]].ctx->lanes].push_back(a);
    size_t gi = 0;
    for (auto& kv : byG) {
      GroupDesc& g = d.groups[gi++];
      const int R = rollouts_per_block(g.G, g.dims);
      std::vector<int> order = kv.second;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const mppi_ctx* cx = reqs[active[it][x]].ctx;
        const mppi_ctx* cy = reqs[active[it][y]].ctx;
        return (long)cx->H * cx->m->host.nsub * cx->m->host.nb > (long)cy->H * cy->m->host.nsub * cy->m->host.nb;
      });
      auto* w = reinterpret_cast<int2*>(h + g.work_off);
      int k = 0;
      for (int a : order)
        for (int n0 = 0; n0 < reqs[active[it][a]].ctx->N; n0 += R) w[k++] = make_int2(a, n0);
    }
  }
  r->pending = true;  // event recorded after the last kernel reading the tables
  if (ns > 0) {
    hipLaunchKernelGGL(stage_kernel, dim3(2 * ns), dim3(64), 0, s, reinterpret_cast<StageItem*>(dv));
    HIP_TRY(hipGetLastError());
  }
  if (nt > 0) {
    int k = 0;
    for (auto& kv : pred_groups) {
      int stride = 0, table = 0;
      for (int i : kv.second) {
        const mppi_ctx* c = reqs[i].ctx;
        stride = std::max(stride, group_floats(kv.first, c->E));
        table = std::max(table, body_sched_table_floats(c->m->host.nb, c->nc));
      }
      HIP_TRY(launch_predict_batch(kv.first, (int)kv.second.size(), reinterpret_cast<const PredItem*>(dv + pred_off) + k,
                                   stride, table, s));
      k += (int)kv.second.size();
    }
    hipLaunchKernelGGL(shift_batch_kernel, dim3(nt), dim3(kShiftThreads), 0, s, reinterpret_cast<const ShiftItem*>(dv + shift_off));
    HIP_TRY(hipGetLastError());
  }
  int ci = 0;
  for (int it = 0; it < Imax; ++it) {
    IterDesc& d = iters[it];
    auto* di = reinterpret_cast<const DevInst*>(dv + d.inst_off);
    const int n_groups = (int)d.groups.size();
    const int n_fork = (fork && fork->n_aux > 0 && n_groups > 1) ? std::min(fork->n_aux, n_groups - 1) : 0;
    if (n_fork > 0) {
      HIP_TRY(hipEventRecord(fork->ev_fork, s));
      for (int j = 0; j < n_fork; ++j) HIP_TRY(hipStreamWaitEvent(fork->aux[j], fork->ev_fork, 0));
    }
    for (int k = 0; k < n_groups; ++k) {
      const GroupDesc& g = d.groups[k];
      const hipStream_t gs = (n_fork > 0 && k > 0) ? fork->aux[(k - 1) % n_fork] : s;
      auto* w = reinterpret_cast<const int2*>(dv + g.work_off);
      if (persistent && counters && ci < n_counters)
        HIP_TRY(launch_persistent(g.G, g.n_items, di, w, g.dims, counters + ci++, gs));
      else
        HIP_TRY(launch_rollout(g.G, g.n_items, di, w, g.dims, gs));
    }
    for (int j = 0; j < n_fork; ++j) {
      HIP_TRY(hipEventRecord(fork->ev_join[j], fork->aux[j]));
      HIP_TRY(hipStreamWaitEvent(s, fork->ev_join[j], 0));
    }
    HIP_TRY(launch_updates(reinterpret_cast<const DevUpdate*>(dv + d.up_off),
                           reinterpret_cast<const UpdateOut*>(dv + d.out_off), d.upd, s));
  }
  HIP_TRY(hipEventRecord(r->ev, s));
  return MPPI_OK;
}

// ---------------------------------------------------------------------------
// serving: continuous batching of MPC ticks from many instances
// ---------------------------------------------------------------------------
namespace {
using Clock = std::chrono::steady_clock;
struct SrvReq {
  mppi_ctx* ctx;
  const float* state;
  const float* knots_in;  // a step's warm start; nullptr for a tick
  float* knots_out;
  Clock::time_point t_submit;
  double latency = 0;
  int status = 0;  // 0 pending, 1 on the device, 2 done
  // a tick (mppi_tick): delay in control steps, tau_best (in/out), step info
  int32_t n_delay = 0;
  float* best = nullptr;
  mppi_step_info* info = nullptr;
};
// mode 2: an admitted request between its iterations
struct SrvLive {
  uint64_t ticket;
  BatchReq req;  // req.it0: its next iteration
};
constexpr int kSrvAux = 3;  // most side streams per slot for a launch's rollout groups
struct SrvSlot {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  hipStream_t aux[kSrvAux] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kSrvAux] = {};
  bool busy = false;
  std::vector<uint64_t> tickets;  // mode 2: the ticks whose last iteration the round runs
  unsigned int* counters = nullptr;
  std::vector<SrvLive> live;      // mode 2: the requests admitted to this stream
};
}  // namespace

struct mppi_server {
  mppi_server_cfg cfg{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, SrvReq> reqs;
  std::unordered_map<const mppi_ctx*, int> busy;
  std::vector<SrvSlot> slots;
  std::thread worker;
  std::atomic<bool> stop{false};
  uint64_t next_ticket = 1;
  std::string error;
  int64_t launched_batches = 0, launched_requests = 0;
  int live_n = 0;  // mode 2: admitted requests not yet complete
  int in_launch = 0;  // modes 0 and 1: requests taken from the queue, their stream not yet marked busy
  int n_aux = 0;   // side streams per slot
  // mode 2, several slots (worker thread only): the slot of each rollout lane key
  // (robot type) and the key owning each slot (kNoOwner: none; keys may be negative)
  std::map<int, int> key_slot;
  std::vector<int> slot_owner;
};

// Mode 2 with several slots: each rollout lane key (robot type) claims a slot
// that no type owns yet when it first appears (once every slot is owned, later
// types share them in turn), and its requests go there, so a slot's rounds never
// wait for a longer kind of rollout.  Slots that no type owns take one type at a
// time (that of their requests in flight, any type once empty), so fewer types
// than slots still use all streams without mixing kinds of rollout in a round.
constexpr int kNoOwner = INT_MIN;
static bool slot_takes(mppi_server* S, int si, const mppi_ctx* c) {
  const int n = (int)S->slots.size();
  if (n == 1) return true;
  auto f = S->key_slot.find(c->lanes);
  if (f == S->key_slot.end()) {
    int s = -1;
    for (int i = 0; i < n && s < 0; ++i)
      if (S->slot_owner[i] == kNoOwner) s = i;
    if (s >= 0)
      S->slot_owner[s] = c->lanes;
    else
      s = (int)S->key_slot.size() % n;
    f = S->key_slot.emplace(c->lanes, s).first;
  }
  if (f->second == si) return true;
  if (S->slot_owner[si] != kNoOwner) return false;
  const SrvSlot& sl = S->slots[si];
  return sl.live.empty() || sl.live.front().req.ctx->lanes == c->lanes;
}

// Side streams per slot.  The runtime maps streams onto a few hardware queues
// (GPU_MAX_HW_QUEUES, 4 by default) and two streams on one queue run in order.
// A single slot forks its rollout groups onto the remaining queues.  With
// several slots, side streams end up sharing queues with other slots' streams
// and each slot's joins then wait behind the others' kernels (measured several
// times slower), so they fork nothing.
static int server_side_streams(int n_streams) {
  if (n_streams != 1) return 0;
  int hwq = 4;
  if (const char* e = std::getenv("GPU_MAX_HW_QUEUES")) {
    const int v = std::atoi(e);
    if (v > 0) hwq = v;
  }
  return std::max(0, std::min(kSrvAux, hwq - 1));
}

static void server_fail(mppi_server* S) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->error = g_err.empty() ? "launch failed" : g_err;
  S->stop = true;
}

// Marks the tickets of a slot whose event has fired as done.
static void server_retire(mppi_server* S, SrvSlot& sl) {
  const auto now = Clock::now();
  std::lock_guard<std::mutex> lk(S->mu);
  for (uint64_t t : sl.tickets) {
    auto it = S->reqs.find(t);
    if (it == S->reqs.end()) continue;
    it->second.status = 2;
    it->second.latency = std::chrono::duration<double>(now - it->second.t_submit).count();
    S->busy.erase(it->second.ctx);
  }
  sl.tickets.clear();
  sl.busy = false;
}

// 1: the slot's launches have finished; 0: still running; -1: the device
// reported an error (the server stops with it).
static int slot_finished(mppi_server* S, SrvSlot& sl) {
  const hipError_t e = hipEventQuery(sl.ev);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  fail(MPPI_EDEVICE, std::string("hipEventQuery: ") + hipGetErrorString(e));
  server_fail(S);
  return -1;
}

static ForkStreams fork_of(const mppi_server* S, const SrvSlot& sl) {
  return ForkStreams{sl.aux, S->n_aux, sl.ev_fork, sl.ev_join};
}

static BatchReq batch_req_of(const SrvReq& r) {
  if (r.best)  // a tick: its prefix runs first, then the iterations read x0 and the nominal in place
    return BatchReq{r.ctx, r.state, nullptr, r.knots_out, r.best, r.info, r.n_delay, true};
  return BatchReq{r.ctx, r.state, r.knots_in, r.knots_out};
}

// Mode 2, iteration-level batching: each stream runs rounds back to back; a
// round runs ONE iteration of every request admitted to that stream (the
// prefixes of the requests admitted at that round first).  Pending requests join
// their stream's next round (with several streams, the stream of their robot
// type, slot_takes) and leave after their last iteration, so nothing waits for the
// rest of a batch to finish and short rollouts do not wait for long ones.  A
// request stays on its stream, which orders its iterations.
static void server_loop_rounds(mppi_server* S) {
  (void)hipSetDevice(S->device);
  std::vector<BatchReq> batch;
  while (!S->stop.load()) {
    bool progressed = false;
    for (int si = 0; si < (int)S->slots.size(); ++si) {
      SrvSlot& sl = S->slots[si];
      if (sl.busy) {
        const int f = slot_finished(S, sl);
        if (f < 0) return;
        if (f == 0) continue;
        server_retire(S, sl);
        progressed = true;
      }
      int admitted = 0;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto it = S->pending.begin(); it != S->pending.end() && S->live_n < S->cfg.max_batch;) {
          SrvReq& r = S->reqs[*it];
          if (S->busy.count(r.ctx) || !slot_takes(S, si, r.ctx)) { ++it; continue; }
          S->busy[r.ctx] = 1;
          r.status = 1;
          BatchReq b = batch_req_of(r);
          if (b.tick && !b.knots_out) b.knots_out = b.ctx->pred_knots;  // as mppi_tick
          sl.live.push_back(SrvLive{*it, b});
          ++admitted;
          ++S->live_n;
          it = S->pending.erase(it);
        }
      }
      if (sl.live.empty()) continue;
      batch.clear();
      for (auto& l : sl.live) {
        BatchReq b = l.req;
        b.n_it = 1;
        batch.push_back(b);
      }
      mppi_status st;
      {
        std::lock_guard<std::mutex> lk(g_mu);
        const ForkStreams fk = fork_of(S, sl);
        st = launch_batch_dynamic(batch, sl.counters, 64 * 5, S->cfg.persistent != 0, sl.stream, &fk);
      }
      if (st == MPPI_OK && hipEventRecord(sl.ev, sl.stream) != hipSuccess) st = MPPI_EDEVICE;
      if (st != MPPI_OK) {
        server_fail(S);
        return;
      }
      std::lock_guard<std::mutex> lk(S->mu);
      size_t k = 0;
      for (auto& l : sl.live) {
        if (++l.req.it0 == l.req.ctx->I) {
          sl.tickets.push_back(l.ticket);
          --S->live_n;
        } else {
          sl.live[k++] = l;
        }
      }
      sl.live.resize(k);
      sl.busy = true;
      S->launched_batches += 1;
      S->launched_requests += admitted;
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

static void server_loop(mppi_server* S) {
  (void)hipSetDevice(S->device);
  std::vector<BatchReq> batch;
  while (!S->stop.load()) {
    bool progressed = false;
    for (auto& sl : S->slots) {
      if (!sl.busy) continue;
      const int f = slot_finished(S, sl);
      if (f < 0) return;
      if (f == 0) continue;
      server_retire(S, sl);
      progressed = true;
    }
    for (auto& sl : S->slots) {
      if (sl.busy) continue;
      batch.clear();
      {
        std::lock_guard<std::mutex> lk(S->mu);
        for (auto it = S->pending.begin(); it != S->pending.end() && (int)batch.size() < S->cfg.max_batch;) {
          SrvReq& r = S->reqs[*it];
          if (S->busy.count(r.ctx)) { ++it; continue; }
          S->busy[r.ctx] = 1;
          r.status = 1;
          batch.push_back(batch_req_of(r));
          sl.tickets.push_back(*it);
          it = S->pending.erase(it);
        }
        S->in_launch += (int)batch.size();  // seen by drain until the slot is marked busy
      }
      if (batch.empty()) continue;
      mppi_status st = MPPI_OK;
      if (S->cfg.mode == 1) {
        for (auto& b : batch) {
          if (b.best_out)
            st = mppi_tick(b.ctx, b.state, b.n_delay, b.best_out, b.knots_out, b.info_out, nullptr, sl.stream);
          else
            st = mppi_step(b.ctx, b.state, b.knots_in, b.knots_out, nullptr, nullptr, nullptr, sl.stream);
          if (st != MPPI_OK) break;
        }
      } else {
        for (auto& b : batch)  // as mppi_tick: a tick without a nominal output writes it where the shift read
          if (b.tick && !b.knots_out) b.knots_out = b.ctx->pred_knots;
        if (st == MPPI_OK) {
          std::lock_guard<std::mutex> lk(g_mu);
          const ForkStreams fk = fork_of(S, sl);
          st = launch_batch_dynamic(batch, sl.counters, 64 * 5, S->cfg.persistent != 0, sl.stream, &fk);
        }
      }
      if (st == MPPI_OK && hipEventRecord(sl.ev, sl.stream) != hipSuccess) st = MPPI_EDEVICE;
      if (st != MPPI_OK) {
        server_fail(S);
        break;
      }
      {
        std::lock_guard<std::mutex> lk(S->mu);  // drain and stats read these
        S->in_launch -= (int)batch.size();
        sl.busy = true;
        S->launched_batches += 1;
        S->launched_requests += (int64_t)batch.size();
      }
      progressed = true;
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

extern "C" mppi_status mppi_server_create(const mppi_server_cfg* cfg, mppi_server** out) {
  if (!cfg || !out) return fail(MPPI_EINVAL, "null argument");
  if (cfg->n_streams < 1 || cfg->n_streams > 8) return fail(MPPI_EINVAL, "n_streams must be in 1..8");
  if (cfg->max_batch < 1 || cfg->max_pending < 1) return fail(MPPI_EINVAL, "max_batch and max_pending must be >= 1");
  if (cfg->mode < 0 || cfg->mode > 2)
    return fail(MPPI_EINVAL, "mode must be 0 (batched), 1 (plain) or 2 (iteration-level)");
  auto S = std::make_unique<mppi_server>();
  S->cfg = *cfg;
  HIP_TRY(hipGetDevice(&S->device));
  S->slots.resize(cfg->n_streams);
  S->slot_owner.assign(cfg->n_streams, kNoOwner);
  S->n_aux = cfg->mode == 1 ? 0 : server_side_streams(cfg->n_streams);
  for (auto& sl : S->slots) {
    HIP_TRY(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    HIP_TRY(hipMalloc(&sl.counters, 64 * 5 * sizeof(unsigned int)));
    HIP_TRY(hipEventCreateWithFlags(&sl.ev_fork, hipEventDisableTiming));
    for (int j = 0; j < S->n_aux; ++j) {
      HIP_TRY(hipStreamCreateWithFlags(&sl.aux[j], hipStreamNonBlocking));
      HIP_TRY(hipEventCreateWithFlags(&sl.ev_join[j], hipEventDisableTiming));
    }
  }
  S->worker = std::thread(cfg->mode == 2 ? server_loop_rounds : server_loop, S.get());
  *out = S.release();
  return MPPI_OK;
}

extern "C" mppi_status mppi_server_submit(mppi_server* S, mppi_ctx* c, const float* d_state, const float* d_knots_in,
                                          float* d_knots_out, uint64_t* ticket) {
  if (!S || !c || !d_state || !d_knots_in || !d_knots_out || !ticket) return fail(MPPI_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(MPPI_EDEVICE, "server stopped: " + S->error);
  if ((int)S->pending.size() >= S->cfg.max_pending) return fail(MPPI_ENOSLOT, "pending queue full");
  const uint64_t t = S->next_ticket++;
  S->reqs[t] = SrvReq{c, d_state, d_knots_in, d_knots_out, Clock::now()};
  S->pending.push_back(t);
  *ticket = t;
  S->cv.notify_one();
  return MPPI_OK;
}

extern "C" mppi_status mppi_server_submit_tick(mppi_server* S, mppi_ctx* c, const float* d_state_meas,
                                               int32_t n_delay, float* d_best, float* d_knots_out,
                                               mppi_step_info* d_info, uint64_t* ticket) {
  if (!S || !c || !d_state_meas || !d_best || !ticket) return fail(MPPI_EINVAL, "null argument");
  if (n_delay < 0 || n_delay > c->H) return fail(MPPI_EINVAL, "n_delay must be in 0..horizon");
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return fail(MPPI_EDEVICE, "server stopped: " + S->error);
  if ((int)S->pending.size() >= S->cfg.max_pending) return fail(MPPI_ENOSLOT, "pending queue full");
  const uint64_t t = S->next_ticket++;
  SrvReq r{c, d_state_meas, nullptr, d_knots_out, Clock::now()};
  r.n_delay = n_delay;
  r.best = d_best;
  r.info = d_info;
  S->reqs[t] = r;
  S->pending.push_back(t);
  *ticket = t;
  S->cv.notify_one();
  return MPPI_OK;
}

extern "C" mppi_status mppi_server_poll(mppi_server* S, uint64_t ticket, int32_t* done, double* latency_s) {
  if (!S || !done) return fail(MPPI_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(MPPI_EINVAL, "unknown ticket");
  *done = it->second.status == 2 ? 1 : 0;
  if (*done) {
    if (latency_s) *latency_s = it->second.latency;
    S->reqs.erase(it);
  }
  if (S->stop && !S->error.empty()) return fail(MPPI_EDEVICE, "server stopped: " + S->error);
  return MPPI_OK;
}

extern "C" mppi_status mppi_server_drain(mppi_server* S, double timeout_s) {
  if (!S) return fail(MPPI_EINVAL, "null server");
  const auto t0 = Clock::now();
  for (;;) {
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stop && !S->error.empty()) return fail(MPPI_EDEVICE, "server stopped: " + S->error);
      bool idle = S->pending.empty() && S->live_n == 0 && S->in_launch == 0;
      for (auto& sl : S->slots) idle = idle && !sl.busy;
      if (idle) return MPPI_OK;
    }
    if (std::chrono::duration<double>(Clock::now() - t0).count() > timeout_s) return fail(MPPI_EBUSY, "drain timed out");
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
}

extern "C" mppi_status mppi_server_stats(mppi_server* S, int64_t* batches, int64_t* requests) {
  if (!S) return fail(MPPI_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  if (batches) *batches = S->launched_batches;
  if (requests) *requests = S->launched_requests;
  return MPPI_OK;
}

extern "C" mppi_status mppi_server_destroy(mppi_server* S) {
  if (!S) return fail(MPPI_EINVAL, "null server");
  S->stop = true;
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);  // the side streams join the slot's stream
    for (int j = 0; j < kSrvAux; ++j)
      if (sl.aux[j]) (void)hipStreamSynchronize(sl.aux[j]);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.ev_fork) (void)hipEventDestroy(sl.ev_fork);
    if (sl.counters) (void)hipFree(sl.counters);
    for (int j = 0; j < kSrvAux; ++j) {
      if (sl.ev_join[j]) (void)hipEventDestroy(sl.ev_join[j]);
      if (sl.aux[j]) (void)hipStreamDestroy(sl.aux[j]);
    }
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete S;
  return MPPI_OK;
}
