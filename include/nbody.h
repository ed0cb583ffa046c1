/*
 * nbody.h -- C ABI of the MI355X (gfx950) gravitational octree library.
 *
 * The library computes the gravitational acceleration of Eq. 1 of Miki,
 * "Gravitational octree code performance evaluation on Volta GPU" (CPC
 * 2019), a_i = sum_{j != i} G m_j (r_j - r_i) / (|r_j - r_i|^2 + eps^2)^(3/2),
 * with the tree method of that paper's Sec. 1: an octree of Morton-sorted
 * particles, monopole moments of every cell (total mass and centre of mass,
 * the "calcNode" function of Sec. 2.2), and a walk in which a group of
 * particles shares one interaction list built with the acceleration
 * multipole acceptance criterion (MAC) of Eq. 2,
 *     G m_J / d^2 (b_J / d)^2 <= delta_acc |a_old|.
 * It also advances particles with a kick-drift-kick leapfrog.
 *
 * Conventions for every entry point
 *  - All particle arrays are DEVICE pointers to contiguous arrays indexed by
 *    the caller's particle order ("caller order"), structure of arrays.
 *    They are owned by the caller and must stay valid until the work
 *    enqueued on the context's stream has finished.
 *  - All work is enqueued on the HIP stream given to nbody_create and the
 *    call returns without waiting, except the functions marked BLOCKING.
 *  - The library allocates no device memory after nbody_bind_workspace: all
 *    scratch lives in the caller-owned workspace.
 *  - Return values are nbody_status codes. Argument errors are returned
 *    directly. Errors found by kernels (non-finite input, overflow of the
 *    walk's frontier buffer) are latched in a device status word, reported
 *    by nbody_sync and by every later call on the context ("sticky").
 *  - No C++ exception crosses this interface. Not thread-safe per context.
 */
#ifndef NBODY_H
#define NBODY_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBODY_ABI_VERSION 4

typedef int32_t nbody_status;
enum {
  NBODY_OK = 0,
  NBODY_EINVAL = -1,     /* bad argument (null pointer, eps <= 0, ...) */
  NBODY_ENOMEM = -2,     /* workspace missing or too small for n */
  NBODY_EHIP = -3,       /* a HIP runtime call failed */
  NBODY_EOVERFLOW = -4,  /* walk frontier overflowed even on the retry (sticky) */
  NBODY_ENOTREE = -5,    /* calc_acc/refit/export before build_tree */
  NBODY_ENONFINITE = -6, /* NaN or Inf in particle input (sticky) */
  NBODY_ECORRUPT = -7    /* a kernel's consistency check failed (sticky) */
};

/* Method parameters.
 *  G, eps      : Eq. 1 constants; eps > 0 (softening, removes the j == i term).
 *  delta_acc   : Eq. 2 accuracy parameter, >= 0. 0 makes the walk exact
 *                (equal to direct summation up to FP32 rounding).
 *  leaf_max    : a cell holding more than leaf_max particles is split
 *                (until level 21); 1 <= leaf_max <= group_max.
 *  group_max   : largest i-group (particles sharing one interaction list);
 *                1 <= group_max <= 64.
 *  compensated : 0 plain FP32 accumulation; 1 compensated (Neumaier) sum.
 *  order       : group queue order of the walk: 0 group (Morton) order;
 *                1 longest expected work first, estimated from the group's
 *                size and its members' previous list lengths; 2 by the
 *                learned cost model (nbody_set_cost_model; plain until one is
 *                installed); 3 by the per-group log2 interaction counts the
 *                last ordered walk recorded (NBODY_X_TARGET): the true costs
 *                when the same groups of the same tree are walked again, an
 *                ideal order for measurements. Orders 1-3 also record the
 *                per-group features and targets of the cost model
 *                (NBODY_X_FEAT, NBODY_X_TARGET). The order never changes the
 *                results (bit-identical). nbody_set_order changes it later.
 *  frontier_cap: cells per wavefront in the walk's candidate stack (power
 *                of two >= 64; 0 = the cell capacity rounded up to a power
 *                of two, at most 16384, which no tree can fill: the stack
 *                holds at most 512 cells per level). A group whose stack
 *                outgrows a smaller cap is walked again by a few wavefronts
 *                with a 16384-cell stack, so the results never depend on it.
 *  list_tile   : interaction-list entries held in LDS per wavefront before a
 *                flush (multiple of 64, 64..2048; 0 = 192).
 *  waves_per_cu: resident wavefronts per compute unit of the persistent walk
 *                (1..32; 0 = 32).
 *  checks      : 0 none; 1 also record, per group, an order-independent hash
 *                of the identities of its interaction-list entries
 *                (NBODY_X_GHASH), for bit-exact checks of every MAC decision.
 *  group_merge : 0 the i-groups are the group cells; 1 consecutive sibling
 *                group cells are joined, in octant order, while the joined
 *                count stays within group_max (fewer, fuller groups, hence
 *                fewer interaction lists; results change only through the
 *                grouping). In a batch (nbody_set_systems) only siblings
 *                within one system are joined: a group never spans systems.
 *  walk_split  : wavefronts sharing one group's interaction list: 0 chosen
 *                per walk from the queued group count q and the walk's
 *                wavefront count w (4 if q < 2w, 2 if q < 4w, else 1), or
 *                1, 2, 4 fixed (1 whenever q > 4w).
 *                A group's list is cut into blocks of 64 entries in
 *                traversal order and each lane keeps 4 FP32 partial sums,
 *                block b adding into sum b mod 4, which are added in that
 *                order at the end; with k wavefronts per group, wavefront j
 *                adds the blocks b with b mod k == j and a second kernel
 *                adds the sums. Results are bit-identical for every value.
 *                The compensated sum (compensated = 1) is never split.
 *  calcnode_sync: how the moment pass ("calcNode", Sec. 2.2) waits for each
 *                tree level's children before their parents (App. A):
 *                0 = library default (1); 1 = one kernel launch per level;
 *                2 = one persistent launch whose workgroups meet at a
 *                lock-free grid barrier (Xiao and Feng 2010) between levels.
 *                Results are bit-identical for every value.
 */
typedef struct {
  float G;
  float eps;
  float delta_acc;
  int32_t leaf_max;
  int32_t group_max;
  int32_t compensated;
  int32_t order;
  int32_t frontier_cap;
  int32_t list_tile;
  int32_t waves_per_cu;
  int32_t checks;
  int32_t group_merge;
  int32_t walk_split;
  int32_t calcnode_sync;
} nbody_params;

typedef struct nbody_ctx nbody_ctx; /* opaque; one per HIP stream */

/* Integration state (all arrays device, caller order, length n).
 * x, y, z: FP64 positions; vx, vy, vz: FP32 velocities; m: FP32 masses;
 * ax, ay, az: FP32 accelerations of the last force evaluation (they are the
 * a_old of Eq. 2 and are overwritten by each step); t: simulation time
 * (host); dt: step length (the longest step dt_max with block steps);
 * have_acc: 0 if ax..az are not yet valid (the first step then runs a
 * bootstrap force evaluation first); rebuild_interval: rebuild the tree
 * every k steps (k >= 1), or 0 to let the library choose by the measured
 * build and walk times (nbody_rebuild_decide).
 *
 * Individual block time steps (the paper's integration, Sec. 1): with
 * level != NULL particle i steps by dt * 2^-level[i]. level (int8, device)
 * is set from the accelerations when have_acc == 0 and otherwise read as
 * given (values outside [level_min, level_max] latch NBODY_ECORRUPT); a new
 * level is the smallest k >= level_min, allowed by the current time, with
 * dt 2^-k <= sqrt(2 eta eps / |a|) (eta > 0), at most level_max (<= 10).
 * tick: time since the start in units of dt * 2^-10 (host; must be >= 0;
 * advanced with t by nbody_step).
 *
 * integrator: 0 kick-drift-kick leapfrog; 1 the second-order Runge-Kutta
 * method in predict / correct form named in Sec. 2.2 (Heun's method, global
 * steps only: level must be NULL): x_p = x + v dt (FP64), v_p = v + a dt
 * (FP32); a_p = walk at x_p (a_old = a); x += (v + v_p) dt/2 (FP64),
 * v += (a + a_p) dt/2 (FP32); a = walk at the new x (a_old = a_p). Two force
 * evaluations per step; the tree is rebuilt (or refitted) for the first and
 * refitted for the second. */
typedef struct {
  int64_t n;
  double *x, *y, *z;
  float *vx, *vy, *vz;
  float *m;
  float *ax, *ay, *az;
  double t;
  double dt;
  int32_t have_acc;
  int32_t rebuild_interval;
  int8_t *level;
  double eta;
  int32_t level_min, level_max;
  int64_t tick;
  int32_t integrator;
} nbody_state;

/* Statistics (host struct filled by nbody_get_stats, BLOCKING).
 *  list_entries, interactions: of the last walk (interaction = one pair of a
 *  group member and a list entry);
 *  t_build_ms, t_walk_ms: latest measured tree build / walk kernel time;
 *  walk_ms_sum/walk_calls, build_ms_sum/build_calls, entries_sum and
 *  interactions_sum: totals since the last nbody_timing call (HIP events on
 *  the context's stream around each walk launch and each build);
 *  queued: groups walked by the last walk; active: particles whose step
 *  ended in the last block step; queued_sum, ngroup_sum: groups walked and
 *  groups present, summed over the walks counted in walk_calls; retried:
 *  groups of the last walk that outgrew frontier_cap and were walked again. */
typedef struct {
  int64_t n, ncell, ngroup;
  int64_t list_entries;
  int64_t interactions;
  int64_t steps, rebuilds;
  double t_build_ms, t_walk_ms;
  double walk_ms_sum;
  int64_t walk_calls;
  double build_ms_sum;
  int64_t build_calls;
  int64_t entries_sum;
  int64_t interactions_sum;
  int64_t queued, active;
  int64_t queued_sum, ngroup_sum;
  int64_t retried;
} nbody_stats;

/* What nbody_export copies (element type, length). */
enum {
  NBODY_X_KEYS = 1,      /* uint64[n]  sorted Morton keys */
  NBODY_X_PERM = 2,      /* uint32[n]  sorted position -> caller index */
  NBODY_X_LEVEL = 3,     /* int32[ncell] */
  NBODY_X_PBEGIN = 4,    /* uint32[ncell] first sorted particle of a cell */
  NBODY_X_PCOUNT = 5,    /* uint32[ncell] */
  NBODY_X_FCHILD = 6,    /* int32[ncell] first child (-1 for a leaf) */
  NBODY_X_NCHILD = 7,    /* int32[ncell] */
  NBODY_X_PARENT = 8,    /* int32[ncell] (-1 for the root) */
  NBODY_X_NODE = 9,      /* float32[ncell][4]: com x, y, z, b^2 */
  NBODY_X_MQ = 10,       /* float32[ncell][2]: m32, q = G m32 b^2 */
  NBODY_X_MOM64 = 11,    /* float64[ncell][4]: M, Sx, Sy, Sz */
  NBODY_X_GBEGIN = 12,   /* uint32[ngroup] */
  NBODY_X_GCOUNT = 13,   /* uint32[ngroup] */
  NBODY_X_GBOX = 14,     /* float32[ngroup][8]: lo xyz, dA, hi xyz, amin */
  NBODY_X_GENTRIES = 15, /* uint32[ngroup] list entries of the last walk */
  NBODY_X_GHASH = 16,    /* uint64[ngroup] order-independent entry hash */
  NBODY_X_XYZM = 17,     /* float32[n][4] sorted positions and masses */
  NBODY_X_BOX = 18,      /* float64[4]: root cube lo x, y, z, side L */
  NBODY_X_QUEUE = 19,    /* uint32[queued] groups walked by the last walk, in order */
  NBODY_X_FEAT = 20,     /* float32[ngroup][4] cost-model features (orders 1, 2;
                            set for the groups of the last walk's queue) */
  NBODY_X_TARGET = 21,   /* float32[ngroup] log2 interactions (groups of the last walk) */
  NBODY_X_PRED = 22,     /* float32[ngroup] the model's prediction (order 2) */
  NBODY_X_SYSBOX = 23,   /* float64[n_sys][4] batch: each system's root cube lo, L */
  NBODY_X_GROOT = 24,    /* uint32[ngroup] batch: each group's walk root cell */
  NBODY_X_APRED = 25     /* float32[3][n] integrator 1: a_p of the last step
                            (x, y, z rows, caller order) */
};

int32_t nbody_abi_version(void);
const char *nbody_strerror(nbody_status s);

/* Fill *p with defaults: G = 1, eps = 2^-7, delta_acc = 2^-9, leaf_max 16,
 * group_max 64, compensated 0, order 0, checks 0, group_merge 1 and the
 * autotunable sizes 0. */
nbody_status nbody_params_default(nbody_params *p);

/* Create a context bound to `hip_stream` (a hipStream_t, NULL = default
 * stream) on the current device. Validates *p (see nbody_params). */
nbody_status nbody_create(const nbody_params *p, void *hip_stream,
                          nbody_ctx **out);
void nbody_destroy(nbody_ctx *ctx);

/* Bytes of device workspace needed for up to n_max particles. BLOCKING
 * only in the sense that it queries the device's compute-unit count. */
nbody_status nbody_workspace_query(const nbody_params *p, int64_t n_max,
                                   size_t *bytes);

/* Bind caller-owned device memory (>= nbody_workspace_query bytes, 256-byte
 * aligned) for up to n_max particles. The library keeps no other device
 * state; rebinding drops the tree. */
nbody_status nbody_bind_workspace(nbody_ctx *ctx, void *dev_ptr, size_t bytes,
                                  int64_t n_max);

/* Tree pipeline of Sec. 1 / Sec. 2.2 for n particles (1 <= n <= n_max):
 * root cube and 63-bit Morton keys, stable radix sort, level-order octree
 * (leaves hold at most leaf_max particles, or sit at level 21), i-groups,
 * and the monopole moments of every cell ("calcNode"). Inputs are FP32
 * positions and masses in caller order (masses >= 0). */
nbody_status nbody_build_tree(nbody_ctx *ctx, int64_t n, const float *x,
                              const float *y, const float *z, const float *m);

/* New positions/masses, same topology: recompute the moments and group
 * boxes on the existing tree (the paper rebuilds the tree only every few
 * steps, Sec. 4.1, while calcNode runs every step). */
nbody_status nbody_refit(nbody_ctx *ctx, const float *x, const float *y,
                         const float *z, const float *m);

/* Group-wise tree walk: accelerations of Eq. 1 under the MAC of Eq. 2 for
 * every particle, written in caller order to ax, ay, az. a_old (caller
 * order) is the previous acceleration used by Eq. 2; pass NULL for all
 * three to run the bootstrap walk, which accepts a cell iff its distance to
 * the group exceeds twice its size b_J. Needs a tree (ENOTREE). */
nbody_status nbody_calc_acc(nbody_ctx *ctx, const float *ax_old,
                            const float *ay_old, const float *az_old,
                            float *ax, float *ay, float *az);

/* nbody_calc_acc that also writes the potential of every particle (caller
 * order, FP32) from the same interaction lists: phi_i = -G sum over the
 * entries j of m_j / (r_ij^2 + eps^2)^(1/2), the particle's own entry left
 * out (the softened potential of Eq. 1's force; W = sum_i m_i phi_i / 2 is
 * the potential energy of long-run energy checks). The walk is never split
 * across wavefronts; accelerations are bit-identical to nbody_calc_acc.
 * Needs a tree (ENOTREE); phi must not be NULL. */
nbody_status nbody_calc_acc_pot(nbody_ctx *ctx, const float *ax_old,
                                const float *ay_old, const float *az_old,
                                float *ax, float *ay, float *az, float *phi);

/* Advance the state by n_steps kick-drift-kick leapfrog steps of length
 * st->dt: v += a dt/2 (FP32); x += v dt (FP64); tree rebuild or refit from
 * the FP32 image of x; a = walk(a_old = previous a); v += a dt/2.
 * st->t is advanced on the host.
 * With block steps (st->level != NULL) one step ends at the next step
 * boundary of the finest occupied level: the particles starting a step take
 * their opening half kick, every particle drifts, the groups holding a
 * particle whose step ends are walked, and those particles take the closing
 * half kick and a new level. Only they receive new accelerations. This form
 * BLOCKS at its end to read the time reached (st->tick, st->t). */
nbody_status nbody_step(nbody_ctx *ctx, nbody_state *st, int32_t n_steps);

/* The global-step form of nbody_step (st->level must be NULL) with a fixed
 * rebuild interval (st->rebuild_interval >= 1), each step replayed from a
 * HIP graph: the first call captures a rebuild step and a refit step on a
 * private stream (default priority) and later calls replay them while the
 * state arrays, n, dt, the queue order and the systems stay the same
 * (otherwise they are captured again). Ordered after earlier work on the
 * context's stream, and later work there waits for it. No timing spans and
 * no rebuild controller inside the graph; results bit-identical to
 * nbody_step with the same interval. */
nbody_status nbody_step_graph(nbody_ctx *ctx, nbody_state *st, int32_t n_steps);

/* Eq. 1 by direct O(N^2) summation in FP32 on the GPU (the tree walk's
 * arithmetic calibration and the delta_acc = 0 reference). */
nbody_status nbody_direct(nbody_ctx *ctx, int64_t n, const float *x,
                          const float *y, const float *z, const float *m,
                          float *ax, float *ay, float *az);

/* Eq. 1 by direct summation in FP64 for the n_target particles targets[k]
 * (device int64, caller indices; an index outside [0, n) gives zeros): the
 * accuracy reference of the tree walk (no tree needed). x, y, z, m are FP32
 * (promoted to FP64); pairs j == i are skipped by index. Outputs per target,
 * device FP64: acceleration (ax, ay, az), and when not NULL the scale
 * aabs = sum_j G m_j |r_ij| / (r_ij^2 + eps^2)^(3/2) (the conditioning of the
 * sum, used to normalise errors) and the potential
 * phi = -sum_{j != i} G m_j / (r_ij^2 + eps^2)^(1/2). */
nbody_status nbody_direct64(nbody_ctx *ctx, int64_t n, const float *x,
                            const float *y, const float *z, const float *m,
                            int64_t n_target, const int64_t *targets, double *ax,
                            double *ay, double *az, double *aabs, double *phi);

/* Copy an internal array (see NBODY_X_*) to caller device memory `dst`
 * holding at least `capacity` elements. Returns ENOMEM if too small.
 * Sizes come from nbody_get_stats. */
nbody_status nbody_export(nbody_ctx *ctx, int32_t what, void *dst,
                          int64_t capacity);

/* BLOCKING: synchronise the stream, then fill *out. */
nbody_status nbody_get_stats(nbody_ctx *ctx, nbody_stats *out);

/* BLOCKING: synchronise the stream and return the sticky status. */
nbody_status nbody_sync(nbody_ctx *ctx);

/* BLOCKING: zero the timing totals of nbody_stats; with enable != 0 also
 * accumulate the interaction count of every later walk on the device (one
 * small reduction kernel after each walk). */
nbody_status nbody_timing(nbody_ctx *ctx, int32_t enable);

/* Host-only rebuild rule used by nbody_step when rebuild_interval == 0
 * (the paper tunes the rebuild interval to minimise tree-construction plus
 * gravity time, Sec. 1 and Sec. 4.1). excess_ms is the measured extra walk
 * time of the current tree: each walk adds t_walk (1 - I_ref / I), where,
 * over the groups this walk and the tree's reference walk (its first walk
 * with the acceleration criterion) both took, I is their interactions now and
 * I_ref then (the whole walk is taken to have grown by the same factor; with
 * block steps the groups walked every step are the heavy ones that dominate
 * the walk time). next_excess_ms is the extra time the coming step's walk is
 * expected to add on the current tree (its walk time on a fresh tree, from
 * the last walk of the same step kind, times the growth I / I_ref - 1 of the
 * last walk). allowed is 0 where a rebuild should wait for the step after
 * (see nbody_rebuild_allowed). Returns 1 (rebuild before the coming step)
 * iff steps_since >= max_interval, or allowed and excess_ms + next_excess_ms
 * >= t_build_ms; 0 if steps_since <= 0. For an excess growing linearly per
 * step this rebuilds at the interval that minimises the mean cost per step.
 * nbody_step decides once every earlier walk is measured.
 * Pure function, no device access. */
int32_t nbody_rebuild_decide(double t_build_ms, double excess_ms, double next_excess_ms,
                             int32_t allowed, int32_t steps_since, int32_t max_interval);

/* Host-only: with block time steps (ticks of dt_max 2^-10), may the tree be
 * rebuilt before the step ending at tick `next_tick`? Only if that step is
 * at least as heavy as the one after it (steps of length `step_ticks`): a
 * step's particles are those of the levels ending at its tick, so its kind
 * is the coarsest such level, 10 - min(ctz(tick), 10); rebuilding before the
 * heavier of two consecutive steps gives the fresh tree to the bigger walk
 * (with levels 0..3 occupied: before every second step). Returns 1 or 0.
 * Pure function, no device access. */
int32_t nbody_rebuild_allowed(int64_t next_tick, int64_t step_ticks);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the tree build
 * and force evaluation of nbody_build_tree followed by nbody_calc_acc in one
 * stateless call, on a workspace the library holds in a static device array
 * of 128 MiB per device (enough for n up to about 2^18 at leaf_max 16; the
 * call returns NBODY_ENOMEM when the layout for (p, n) does not fit). It
 * calls no allocator: no context, no events, no host copies; everything is
 * enqueued on hip_stream and the call returns at once. p as for
 * nbody_create; frontier_cap above 256 (or 0) is taken as 256, walk_split,
 * order and calcnode_sync are fixed (none of them changes a result: the
 * accelerations equal those of the context path bit for bit). x, y, z, m:
 * device FP32, caller order, length n; ax_old..az_old: a_old of Eq. 2, or all
 * NULL for the bootstrap criterion; ax..az: device outputs, caller order.
 * status_dev (device int32, may be NULL) receives the device-side status
 * bits of the call (0, or a nonzero word where nbody_sync would report
 * NBODY_EOVERFLOW / NBODY_ENONFINITE / NBODY_ECORRUPT); argument errors are
 * returned directly. All calls on one device share the one array: calls
 * that overlap in time on a device race (serialise them on one stream). */
nbody_status nbody_tree_forces_noalloc(const nbody_params *p, void *hip_stream, int64_t n,
                                       const float *x, const float *y, const float *z,
                                       const float *m, const float *ax_old,
                                       const float *ay_old, const float *az_old, float *ax,
                                       float *ay, float *az, int32_t *status_dev);

/* ---- Cost model of the walk queue (a small MLP: 4 inputs, two tanh layers
 * of `hidden` units, one output; hidden in {8, 16, 32, 64}). It predicts a
 * group's log2 interaction count from NBODY_X_FEAT-style features: log2 of
 * the member count, log2(h + 2^-40) with h half the diagonal of the members'
 * box, log2 of the group mass minus 3x the previous value, and log2(1 + the
 * members' mean list length from their last walk on the current tree; 0 for
 * members not walked since the tree was built). Weights: FP32, row-major
 * output-major, mu[4] is[4] W1[H][4] b1[H] W2[H][H] b2[H] W3[H] b3; the
 * inputs are standardised first, z = (f - mu) * is, with mu, is constants of
 * the model (their gradient entries are 0). The network's output is a
 * correction to the size-based estimate f0 + f3 (log2 count + log2(1 + mean
 * previous list length)): the prediction is y = net(z) + (f0 + f3). All arrays are
 * device memory; feat is [rows][4] FP32, 16-byte aligned. Calls enqueue on
 * the context's stream (they need a bound workspace for scratch). */

/* Number of weights for `hidden`, or -1 if hidden is not supported. */
int64_t nbody_mlp_nparams(int32_t hidden);

/* y[r] = the model's prediction for feat[r] (the network's output plus
 * feat[r][0] + feat[r][3]). */
nbody_status nbody_mlp_forward(nbody_ctx *ctx, int32_t hidden, const float *w,
                               int64_t rows, const float *feat, float *y);

/* grad_loss[0 .. np) = gradient of L = mean_r (y_r - target_r)^2 with
 * respect to w (same layout), grad_loss[np] = L. Deterministic (fixed
 * reduction order). */
nbody_status nbody_mlp_grad(nbody_ctx *ctx, int32_t hidden, const float *w,
                            int64_t rows, const float *feat, const float *target,
                            float *grad_loss);

/* One Adam step (Kingma and Ba 2015), step >= 1, in place on w, m, v. */
nbody_status nbody_mlp_adam(nbody_ctx *ctx, int64_t n_params, float *w,
                            const float *grad, float *m, float *v, int32_t step,
                            float lr, float beta1, float beta2, float eps);

/* BLOCKING: set the standardisation of w from the rows (mean, 1 / standard
 * deviation), then `steps` full-batch Adam steps (beta 0.9, 0.999, eps 1e-8)
 * on the mean squared error, starting from and updating w. loss_out (host,
 * may be NULL) receives the loss before each step. */
nbody_status nbody_costmodel_train(nbody_ctx *ctx, int32_t hidden, float *w,
                                   int64_t rows, const float *feat,
                                   const float *target, int32_t steps, float lr,
                                   float *loss_out);

/* Install (copy) the weights used by order 2; w == NULL removes the model. */
nbody_status nbody_set_cost_model(nbody_ctx *ctx, int32_t hidden, const float *w);

/* Change the queue order (0, 1 or 2, as nbody_params.order). */
nbody_status nbody_set_order(nbody_ctx *ctx, int32_t order);

/* Where nbody_step keeps the state during block steps (Sec. 1 and 4.1: every
 * per-particle pass of a step runs over the tree's sorted order). layout 1:
 * in the tree's key order, gathered from the caller's arrays on entry,
 * permuted at each rebuild and scattered back on exit; 2: in the caller's
 * arrays, reached through the tree's permutation; 0 (the default): 1 for
 * calls of at least 8 steps, else 2 (the gather and scatter cost about what
 * eight steps save). Results are bit-identical in every layout. EINVAL for
 * other values. */
nbody_status nbody_set_step_layout(nbody_ctx *ctx, int32_t layout);

/* ---- Batches of independent systems in one tree (one sort, one build,
 * one persistent walk for all of them). offsets (host, n_sys + 1 entries,
 * offsets[0] = 0, strictly increasing: no empty system) give each system's
 * caller-order range; later builds (nbody_build_tree with n = offsets[n_sys],
 * nbody_step) use them. Each system gets its own root cube; its index fills
 * the top r octal digits of the key (r = smallest with 8^r >= n_sys, 0 for
 * one system) above a Morton key of 21 - r levels; cells above level r are
 * always split, groups lie at level r or deeper, and each group's walk
 * starts at its system's root, so no interaction crosses systems. n_sys = 1
 * returns to a single system. BLOCKING (copies the offsets). */
nbody_status nbody_set_systems(nbody_ctx *ctx, int32_t n_sys, const int64_t *offsets);

#ifdef __cplusplus
}
#endif
#endif
