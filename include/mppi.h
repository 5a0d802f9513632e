/*
 * mppi.h -- C ABI of the MI355X (gfx950) hot path of reference-free
 * sampling-based MPC (Schramm, Fabre, Perrin-Gilbert, Carpentier,
 * arXiv 2511.19204).
 *
 * One call to mppi_step runs the inner loop of the paper's Algorithm 1
 * ("Reference-Free MPPI") for one robot state: I planning iterations of
 *   sample perturbed spline knots  (Alg. 1 sampling step, Sec. III-B noise
 *                                   schedule, eq. vel-clamp),
 *   roll every sample out          (Alg. 1 simulate step: PD tracking of the
 *                                   cubic Hermite reference, eq. hermite_segment
 *                                   and eq. pd-controller; floating-base rigid
 *                                   bodies with soft contact),
 *   score it                       (Sec. IV-A running and terminal costs),
 *   weight and update              (eq. softmax_minmax / eq. omega-weights and
 *                                   eq. update-nominal applied to the knots),
 *   track the best sample          (Sec. III-D).
 * All compute runs in hand-written HIP kernels on the device; the host only
 * validates arguments and enqueues work.
 *
 * Conventions
 *   - Spatial vectors are (angular; linear).
 *   - A floating-base model has body 0 = free base; its state is
 *     q = [p(3), quaternion w,x,y,z (4), joints(n_u)],
 *     v = [base angular velocity (3), base linear velocity (3), joints(n_u)],
 *     the base twist in base coordinates.  A fixed-base model has q = v = joints.
 *   - Every other body carries one revolute joint (joint j of body j + 1, or
 *     body j for a fixed base).  Parents precede children (parent[i] < i).
 *   - Knot arrays are [2][n_knots][n_u] float: positions, then velocities.
 *   - Device pointers are plain hipMalloc'd (or torch) device memory on the
 *     current device; host pointers are read only during the call.
 *   - Calls are asynchronous on the given stream (hipStream_t passed as void*,
 *     NULL = the null stream); outputs are valid once the stream completes.
 *   - Results are a pure function of (model, params, seed, tick, state,
 *     knots_in): independent of batching, launch shape, stream and other work.
 *
 * Errors: every entry point returns an mppi_status.  Argument and shape errors
 * are detected on the host (MPPI_EINVAL); HIP runtime failures give
 * MPPI_EDEVICE; mppi_last_error() returns a thread-local message for the last
 * non-OK status.  Device data is never inspected on the host: non-finite
 * rollouts are counted and given zero weight on the device.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPPI_OK = 0,
  MPPI_EINVAL = -1,
  MPPI_ENOMEM = -2,
  MPPI_EDEVICE = -3,
  MPPI_EBUSY = -4,
  MPPI_ENOSLOT = -5
} mppi_status;

/* Kinematic tree, inertias, actuators and soft contact (host memory, float).
 * The tree is the robot the rollouts simulate (the paper simulates its robots
 * in the Simple simulator; this library integrates them itself, see below). */
typedef struct {
  int32_t n_bodies;          /* 1..64                                          */
  int32_t floating_base;     /* 1: body 0 is a 6-DoF free base; 0: fixed base  */
  const int32_t* parent;     /* [n_bodies], parent[i] < i, -1 = world          */
  const float* axis;         /* [n_bodies][3] unit joint axis in the joint frame */
  const float* R_tree;       /* [n_bodies][9] row-major, joint frame in parent  */
  const float* p_tree;       /* [n_bodies][3] joint frame origin in parent      */
  const float* mass;         /* [n_bodies]                                      */
  const float* com;          /* [n_bodies][3] centre of mass in the body frame  */
  const float* inertia;      /* [n_bodies][6] xx yy zz xy xz yz about the com   */
  const float* q_min;        /* [n_u] joint position bounds                    */
  const float* q_max;        /* [n_u]                                           */
  const float* tau_max;      /* [n_u] actuator torque limits                    */
  const float* kp;           /* [n_u] PD gains                                  */
  const float* kd;           /* [n_u]                                           */
  int32_t n_contacts;        /* 0..32                                           */
  const int32_t* contact_body; /* [n_contacts]                                  */
  const float* contact_pos;  /* [n_contacts][3] point in the body frame         */
  float k_contact;           /* normal spring  N/m  (ground plane z = 0)        */
  float d_contact;           /* normal damper  N s/m                            */
  float mu;                  /* Coulomb friction coefficient                    */
  float eps_fric;            /* friction smoothing velocity  m/s                */
  float gravity;             /* m/s^2, along -z                                 */
  int32_t ee_body;           /* end-effector body for the reaching cost, or -1  */
  float ee_pos[3];           /* end-effector point in that body's frame         */
  int32_t n_substeps;        /* physics steps per control step, >= 1            */
  const float* armature;     /* [n_u] reflected rotor inertia per joint, or NULL (zero) */
} mppi_model_desc;

/* Controller parameters of one MPC instance (the Require line of Alg. 1 plus
 * the cost weights of Sec. IV-A). */
typedef struct {
  int32_t n_samples;         /* N: sampled trajectories per iteration, 1..65536 */
  int32_t horizon;           /* H: control steps per rollout, 1..4096           */
  int32_t n_knots;           /* K: spline knots per joint, 2..64                */
  int32_t n_iters;           /* I: planning iterations per call, 1..64          */
  float dt;                  /* control step, s                                 */
  float lambda;              /* softmax temperature > 0                         */
  int32_t weight_mode;       /* 0: min-max normalised costs, 1: raw costs       */
  int32_t noise_mode;        /* 0: exponential annealing kernel, 1: linear      */
  float scale_q, beta1, beta2; /* mode 0: std = scale_q exp(-(I-i)/(beta1 I) - (K-k)/(beta2 K)) */
  float sigma_lo, sigma_hi;  /* mode 1: std = lo + (hi - lo) k / (K - 1)        */
  int32_t cost_kind;         /* 0: end-effector height, 1: locomotion           */
  float w_h, w_or, w_q, w_cv, w_cf, w_eff, w_H; /* locomotion weights           */
  float w_ee, w_tau;         /* end-effector weights                           */
  float z_des;               /* desired base (or end-effector) height           */
  float v_des[3];            /* commanded base velocity (terminal target)       */
  const float* f0z;          /* [n_contacts] reference normal force per point   */
  const float* q0_cost;      /* [n_u] reference joint configuration             */
  int32_t spline_mode;       /* control parameterization (spline ablation, Sec. V):
                              * 0 cubic Hermite: position and velocity knots,
                              *   velocity targets = the spline's derivative;
                              * 1 natural cubic spline through the position
                              *   knots, velocity targets zero;
                              * 2 C1 quadratic spline (zero initial slope)
                              *   through the position knots, velocity targets
                              *   zero.  Modes 1 and 2 sample positions only and
                              *   keep the spline's knot slopes (dq/dt) in the
                              *   velocity block of every knot vector they return. */
  /* Task targets (Sec. IV-A, Tab. cost-weights): */
  float q_des[4];            /* base orientation target R_des as a unit quaternion
                              * (w, x, y, z); the orientation term is w_or times the
                              * squared rotation angle of R_base^T R_des.  All zero
                              * stands for the identity (level base, any yaw 0).  */
  int32_t terminal_z_abs;    /* 0: terminal target p_base(x0) + v_des H dt;
                              * 1: its height is z_terminal instead (jumping)      */
  float z_terminal;
} mppi_params;

/* Task targets that may change between calls (e.g. the height step of the
 * jumping task): the same fields as in mppi_params. */
typedef struct {
  float z_des;
  float v_des[3];
  float q_des[4];
  int32_t terminal_z_abs;
  float z_terminal;
} mppi_targets;

/* Per-call results besides the knots (device memory).  best_iter == 0 and
 * best_sample == 0 mean that no sample improved on the warm start (the
 * "failed to improve" statistic of the best-trajectory ablation). */
typedef struct {
  float S_best;              /* lowest cost simulated in this call (+inf if none) */
  int32_t best_iter;         /* iteration that found it, -1 if none             */
  int32_t n_nonfinite;       /* rollouts with a non-finite cost, all iterations */
  int32_t all_nonfinite_iters; /* iterations whose rollouts were all non-finite  */
  int32_t best_sample;       /* sample index of the best within best_iter (0 = that iteration's nominal), -1 if none */
} mppi_step_info;

typedef struct mppi_model mppi_model;   /* device-resident tree (opaque)       */
typedef struct mppi_ctx mppi_ctx;       /* one MPC instance (opaque)           */

/* Upload a tree.  Validates shapes (parent order, unit axes within 1e-4,
 * positive masses, contact bodies in range).  The model owns its device copy;
 * the caller keeps ownership of desc.  Errors: MPPI_EINVAL, MPPI_EDEVICE. */
mppi_status mppi_model_create(const mppi_model_desc* desc, mppi_model** out);
mppi_status mppi_model_destroy(mppi_model* m);

/* Create an MPC instance on the current device.  Precomputes the noise
 * schedule (Sec. III-B, "precomputed and cached once") in FP64 and stores it as
 * float; allocates the per-sample knot and cost buffers.  The counter-based
 * noise is keyed by seed; the tick counter starts at 0 and advances by one per
 * mppi_step.  The model must outlive the context. */
mppi_status mppi_create(const mppi_model* m, const mppi_params* p, uint64_t seed, mppi_ctx** out);
mppi_status mppi_destroy(mppi_ctx* c);
mppi_status mppi_set_tick(mppi_ctx* c, uint32_t tick);
mppi_status mppi_get_tick(const mppi_ctx* c, uint32_t* tick);

/* Rollout schedule: how the lanes of a wavefront share the rigid-body tree of
 * one rollout (the articulated-body sweeps of the forward dynamics).
 *   MPPI_SCHEDULE_BODY   one lane per body; the tree is swept level by level,
 *                        lanes per rollout = a power of two 4..64 >= n_bodies.
 *   MPPI_SCHEDULE_CHAIN  one lane per kinematic chain of the tree's heavy-path
 *                        decomposition (a body continues its parent's chain when
 *                        it heads the parent's largest subtree); each lane walks
 *                        its chain, lanes per rollout = the next power of two
 *                        >= the number of chains.  Needs at most 8 chains and
 *                        tree depth <= 15 (MPPI_EINVAL otherwise).
 *   MPPI_SCHEDULE_TEAM   the chains of MPPI_SCHEDULE_CHAIN, each on a block of
 *                        4 or 8 lanes: one body per lane for the per-body work,
 *                        and the block's first three lanes together (one
 *                        spatial coordinate each) for the sweeps; lanes per
 *                        rollout = the next power of two >= chains x block.
 *                        Same conditions as the chain schedule, and at most 64
 *                        lanes per rollout.
 * The body and chain schedules and every lane count give bit-identical
 * results; the team schedule evaluates the same formulas with sums taken in
 * another order, so its results differ from theirs by rounding (its own results
 * are deterministic and independent of batching).  A new context uses the body
 * schedule with the smallest lane count that holds the tree; mppi_autotune
 * times all of them.
 * mppi_set_lanes_per_rollout selects the body schedule with `lanes` lanes (0 =
 * the smallest valid count); mppi_get_lanes_per_rollout reports the lane count
 * of the current schedule. */
typedef enum { MPPI_SCHEDULE_BODY = 0, MPPI_SCHEDULE_CHAIN = 1, MPPI_SCHEDULE_TEAM = 2 } mppi_schedule;
mppi_status mppi_set_schedule(mppi_ctx* c, int32_t schedule);
mppi_status mppi_get_schedule(const mppi_ctx* c, int32_t* schedule);
mppi_status mppi_set_lanes_per_rollout(mppi_ctx* c, int32_t lanes);
mppi_status mppi_get_lanes_per_rollout(const mppi_ctx* c, int32_t* lanes);

/* One MPC step (Alg. 1 inner loop, I iterations) from d_state.
 *   d_state      [n_q + n_v] device float, the (predicted) robot state
 *   d_knots_in   [2][K][n_u] device float, warm-start nominal knots
 *   d_knots_out  [2][K][n_u] device float, nominal after I iterations (may alias d_knots_in)
 *   d_best_knots [2][K][n_u] device float or NULL, the best simulated sample
 *   d_info       device mppi_step_info or NULL
 *   d_costs      [I][N] device float or NULL, every rollout cost
 * Uses the context's tick, then advances it.  If every rollout of an
 * iteration is non-finite the nominal is left unchanged for that iteration. */
mppi_status mppi_step(mppi_ctx* c, const float* d_state, const float* d_knots_in, float* d_knots_out,
                      float* d_best_knots, mppi_step_info* d_info, float* d_costs, void* stream);

/* State prediction (Sec. III-E): the state reached from d_state_in
 * [n_q + n_v] after n_steps control steps (0..H) of the trajectory that d_knots
 * [2][K][n_u] defines (its first n_steps actions, PD-tracked with the rollout's
 * own dynamics, soft contact and integrator), written to d_state_out
 * [n_q + n_v] (device; may alias d_state_in).  Errors: MPPI_EINVAL. */
mppi_status mppi_predict(mppi_ctx* c, const float* d_state_in, const float* d_knots, int32_t n_steps,
                         float* d_state_out, void* stream);

/* Warm-start shift (Sec. III-E): d_knots_out [2][K][n_u] = the spline of
 * d_knots_in evaluated at t_k + n_steps dt (value and derivative), with the
 * time clamped to the horizon end so the final action repeats.  n_steps >= 0;
 * the buffers may alias. */
mppi_status mppi_shift_knots(mppi_ctx* c, const float* d_knots_in, int32_t n_steps, float* d_knots_out,
                             void* stream);

/* One control step of Alg. 1 with state prediction and warm start, all on the
 * stream: x_t = predict(d_state_meas, tau_best, n_delay); tau_0 = tau_best
 * shifted by n_delay; then the I iterations of mppi_step from (x_t, tau_0).
 *   d_state_meas [n_q + n_v] device, the last measured state (n_delay control
 *                steps old)
 *   d_best       [2][K][n_u] device, in: tau_best of the previous tick; out: the
 *                best trajectory simulated in this tick (the one to execute)
 *   d_knots_out  [2][K][n_u] device or NULL, the final nominal
 *   d_info       device mppi_step_info or NULL (best_iter == 0 and best_sample
 *                == 0: no sample improved on the shifted previous solution)
 *   d_state_pred [n_q + n_v] device or NULL, the predicted state x_t
 * Uses the context's tick, then advances it.  Errors: MPPI_EINVAL (n_delay
 * outside 0..H, null required pointer), MPPI_EDEVICE. */
mppi_status mppi_tick(mppi_ctx* c, const float* d_state_meas, int32_t n_delay, float* d_best, float* d_knots_out,
                      mppi_step_info* d_info, float* d_state_pred, void* stream);

/* The same for n instances in fused launches (each array has n entries;
 * d_best_knots / d_info entries may be NULL).  Instances may differ in model,
 * N, H, K and I.  Each result equals that instance's own mppi_step. */
mppi_status mppi_step_batch(int32_t n, mppi_ctx* const* ctxs, const float* const* d_states,
                            const float* const* d_knots_in, float* const* d_knots_out,
                            float* const* d_best_knots, mppi_step_info* const* d_infos, void* stream);

/* Process-wide options of batched launches.  persistent = 1 runs each rollout
 * launch of a batch as a persistent grid (one workgroup per resident wavefront
 * slot) whose wavefronts take (instance, sample) work items from a device
 * counter, longest rollouts first; 0 launches one workgroup per work item.
 * Results do not depend on the choice. */
typedef struct {
  int32_t persistent;
} mppi_batch_opts;
mppi_status mppi_set_batch_options(const mppi_batch_opts* o);

/* A fixed batch captured once into a hipGraph (inputs/outputs as in
 * mppi_step_batch, pointers fixed at capture, buffers owned by the caller and
 * alive while the graph is used).  Each mppi_graph_launch is one MPC step of
 * every instance and advances their ticks; it equals mppi_step_batch on the
 * same pointers.  The graph holds kernel nodes only. */
typedef struct mppi_graph mppi_graph;
mppi_status mppi_graph_create(int32_t n, mppi_ctx* const* ctxs, const float* const* d_states,
                              const float* const* d_knots_in, float* const* d_knots_out,
                              float* const* d_best_knots, mppi_step_info* const* d_infos, mppi_graph** out);
mppi_status mppi_graph_launch(mppi_graph* g, void* stream);
mppi_status mppi_graph_destroy(mppi_graph* g);

/* Autotuner: times `reps` steps of the instance from (d_state, d_knots) for the
 * body schedule at each valid lane count, for the chain schedule and for the
 * team schedule (where the tree allows them), and keeps the fastest; results
 * are cached per (model, N, H, K) for the process.  The
 * instance's tick is restored.  Blocks until the timing steps finish.  Writes
 * the chosen lane count to *best_lanes (nullable); mppi_get_schedule tells the
 * schedule. */
mppi_status mppi_autotune(mppi_ctx* c, const float* d_state, const float* d_knots, int32_t reps, void* stream,
                          int32_t* best_lanes);

/* Replace the instance's task targets (cost definition of Sec. IV-A).  The
 * change is one small kernel on `stream` (hipStream_t, NULL = the null stream)
 * that writes the instance's device target block, which the kernels read when
 * they run: work enqueued on `stream` after this call sees the new targets,
 * work before it the old ones, and nothing else waits (no device-wide
 * synchronisation).  Work of the instance on other streams -- a server's
 * streams, graphs launched elsewhere -- is not ordered with the change: order
 * it with events, or change targets while none of the instance's work is in
 * flight.  Launch plans and graphs stay valid and use the targets current when
 * they run.  MPPI_EINVAL for a non-unit orientation target. */
mppi_status mppi_set_targets(mppi_ctx* c, const mppi_targets* t, void* stream);

/* ---- Serving: continuous batching of MPC ticks --------------------------- */

/* A server owns HIP streams and a worker thread.  Submitted ticks wait in a
 * FIFO; one outstanding tick per instance is on the device at a time.
 *  mode 0 (request-level batching): whenever one of the n_streams streams is
 *    free the worker forms a batch of up to max_batch pending ticks and launches
 *    all their iterations as one fused batched step; ticks that arrive while
 *    others run join the next batch, so several batches overlap on the device.
 *  mode 1: the same, with plain per-instance steps (the baseline).
 *  mode 2 (iteration-level batching): each of the n_streams streams runs
 *    rounds back to back; a round launches ONE iteration (Alg. 1) of every tick
 *    admitted to that stream, after the prefixes of the ticks admitted at that
 *    round.  Pending ticks join their stream's next round (up to max_batch
 *    admitted over all streams) and leave after their last iteration.  With
 *    several streams each robot type (instances with the same lanes per
 *    rollout) claims a stream no type owns when it first appears and its ticks
 *    go there, so short rollouts never wait for a round of long ones; a stream
 *    no type owns serves one type at a time (once all are owned, later types
 *    share).
 * With n_streams = 1 in mode 0 or 2, each launch forks its rollout kernels (one
 * per lane count) onto up to three side streams of the server, fewer when
 * GPU_MAX_HW_QUEUES is below 4, so that kernels of different robot types run
 * side by side; with several streams nothing forks.  Streams beyond the
 * process's hardware queue count (GPU_MAX_HW_QUEUES, four unless set before the
 * process first touches the GPU) share queues, whose time-slicing delays every
 * round on them: give each server stream a queue of its own (n_streams plus the
 * caller's busy streams at most GPU_MAX_HW_QUEUES).
 * Each result equals the instance's own mppi_step / mppi_tick (the instance's
 * warm-start knots and noise tick stay on the device).  persistent selects the
 * persistent rollout launch (mppi_batch_opts).  Buffers passed to submit must
 * stay valid until the tick is reported done. */
typedef struct {
  int32_t max_pending;   /* pending ticks beyond which submit returns MPPI_ENOSLOT */
  int32_t n_streams;     /* 1..8 batches (mode 2: rounds) in flight             */
  int32_t max_batch;     /* ticks per batch (mode 2: admitted over all streams) */
  int32_t mode;          /* 0 batched, 1 plain per-instance, 2 iteration-level  */
  int32_t persistent;    /* 1: persistent rollout launches                      */
} mppi_server_cfg;
typedef struct mppi_server mppi_server;
mppi_status mppi_server_create(const mppi_server_cfg* cfg, mppi_server** out);
/* Non-blocking; *ticket identifies the tick.  MPPI_ENOSLOT when the queue is full. */
mppi_status mppi_server_submit(mppi_server* s, mppi_ctx* c, const float* d_state, const float* d_knots_in,
                               float* d_knots_out, uint64_t* ticket);
/* A tick as mppi_tick (state prediction and warm-start shift of Sec. III-E, then
 * the iterations of Alg. 1), served like mppi_server_submit: the measured state
 * d_state_meas is carried n_delay (0..H) control steps along d_best, d_best
 * shifted by n_delay actions is the warm start, and the best trajectory of the
 * iterations replaces d_best (device, [2][K][n_u], owned by the caller).
 * d_knots_out (nominal after the last iteration) and d_info are nullable.  In a
 * batch the prefixes run on the batch's stream before its fused iterations; the
 * result equals the instance's own mppi_tick.  MPPI_EINVAL for a delay outside
 * 0..H, MPPI_ENOSLOT when the queue is full. */
mppi_status mppi_server_submit_tick(mppi_server* s, mppi_ctx* c, const float* d_state_meas, int32_t n_delay,
                                    float* d_best, float* d_knots_out, mppi_step_info* d_info, uint64_t* ticket);
/* *done = 1 once the tick's outputs are complete on the device; then *latency_s is
 * submit-to-completion wall time and the ticket is released. */
mppi_status mppi_server_poll(mppi_server* s, uint64_t ticket, int32_t* done, double* latency_s);
/* Wait (up to timeout_s) until nothing is pending or in flight; MPPI_EBUSY on timeout. */
mppi_status mppi_server_drain(mppi_server* s, double timeout_s);
/* batches: launches so far (mode 2: rounds); requests: ticks they admitted. */
mppi_status mppi_server_stats(mppi_server* s, int64_t* batches, int64_t* requests);
mppi_status mppi_server_destroy(mppi_server* s);

/* ---- Verification entry points (same device code as mppi_step) ---------- */

/* Philox4x32-10 block function: d_ctr [n][4], d_key [n][2] -> d_out [n][4]. */
mppi_status mppi_debug_philox(const uint32_t* d_ctr, const uint32_t* d_key, uint32_t* d_out, int32_t n,
                              void* stream);

/* The perturbed, clipped and clamped knots of every sample of iteration iter
 * at tick `tick` around d_knots_in: d_samples [N][2][K][n_u]. */
mppi_status mppi_debug_samples(mppi_ctx* c, const float* d_knots_in, int32_t iter, uint32_t tick,
                               float* d_samples, void* stream);

/* Accelerations of one physics step of step size dt for n states: PD tracking
 * of (d_qref, d_vref) [n][n_u], soft contact and the linearly implicit terms.
 * d_q [n][n_q], d_v [n][n_v] -> d_qdd [n][n_v]. */
mppi_status mppi_debug_dynamics(const mppi_model* m, int32_t n, const float* d_q, const float* d_v,
                                const float* d_qref, const float* d_vref, float dt, float* d_qdd,
                                void* stream);

/* Roll out given sample knots d_samples [N][2][K][n_u] from d_state:
 * d_costs [N]; d_masks [N][H] (nullable) = contact bitmask at each control step. */
mppi_status mppi_debug_rollouts(mppi_ctx* c, const float* d_state, const float* d_samples, float* d_costs,
                                uint32_t* d_masks, void* stream);

/* Step-by-step record of iteration `iter` of mppi_step at noise tick `tick`,
 * from d_state and the nominal d_knots_in, with mppi_step's own rollout kernel
 * and launch shape (the simulate step of Alg. 1 with the Sec. IV-A costs):
 *   d_trace_map [N] device int32, record slot of sample n or -1 (not recorded)
 *   d_trace     [slots][H + 1][nq + 2 nv + 2] device float: record h < H holds
 *               the state (q, v) at the start of control step h, the
 *               accelerations of its first physics substep (nv), its running
 *               cost and its contact mask (uint32 bits); record H holds the
 *               final state, zero accelerations, the terminal cost and 0
 *   d_samples   [N][2][K][n_u], d_costs [N], d_masks [N][H] device outputs
 * Body schedule only (MPPI_EINVAL otherwise).  Blocks until done. */
mppi_status mppi_debug_trace(mppi_ctx* c, const float* d_state, const float* d_knots_in, int32_t iter, uint32_t tick,
                             const int32_t* d_trace_map, float* d_trace, float* d_samples, float* d_costs,
                             uint32_t* d_masks, void* stream);

/* Weights and update from given costs d_costs [N] and samples d_samples
 * [N][2][K][n_u]: d_knots_out = sum_n w_n sample_n (unchanged d_knots_in if no
 * cost is finite), d_weights [N] (nullable). */
mppi_status mppi_debug_update(mppi_ctx* c, const float* d_costs, const float* d_samples,
                              const float* d_knots_in, float* d_knots_out, float* d_weights, void* stream);

/* ---- Without allocation -------------------------------------------------- */

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the weights
 * and weighted knot update of mppi_debug_update, with the instance's settings
 * passed directly instead of a context, and the update's scratch (per-slice
 * weighted sums, the finished-slice counter, a running-best record) in a fixed
 * device array of the library instead of per-context buffers.
 *   n_samples    N, 1..65536; n_elems E = 2 K n_u, 1..8192
 *   lambda > 0, weight_mode 0 (min-max normalised) or 1 (raw), as in mppi_params
 *   d_costs [N], d_samples [N][E] (16-byte aligned when E is a multiple of 4),
 *   d_knots_in [E]: device inputs; d_knots_out [E] = sum_n w_n sample_n
 *   (d_knots_in unchanged if no cost is finite), d_weights [N] or NULL
 * The array holds 64 x 8192 + 8264 floats (about 2.03 MiB) per device that
 * calls it, kept until the process ends; its address is looked up once per
 * device.  The call allocates nothing and launches two kernels on the stream
 * (a counter reset and the update).  Every call on one device shares that
 * device's array, so calls that overlap on one device race: order them on one
 * stream (or with events).  Errors: MPPI_EINVAL for sizes beyond the maximum,
 * null or misaligned pointers; MPPI_EDEVICE. */
mppi_status mppi_update_noalloc(int32_t n_samples, int32_t n_elems, float lambda, int32_t weight_mode,
                                const float* d_costs, const float* d_samples, const float* d_knots_in,
                                float* d_knots_out, float* d_weights, void* stream);

/* ---- Kernel timing ------------------------------------------------------- */

/* When enabled, mppi_step records three HIP events per iteration on its stream:
 * before the rollout launch, between the rollout and the update launch, and after
 * the update launch.  mppi_profile_read waits for the recorded events, returns the
 * summed rollout and update time (ms) and launch counts since the last read, and
 * recycles the events.  Costs a few microseconds per event; off by default. */
mppi_status mppi_profile_enable(mppi_ctx* c, int32_t on);
mppi_status mppi_profile_read(mppi_ctx* c, double* rollout_ms, int32_t* n_rollout, double* update_ms,
                              int32_t* n_update);

const char* mppi_last_error(void);
const char* mppi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPPI_H */
