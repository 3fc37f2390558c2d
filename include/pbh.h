/*
 * pbh.h -- C ABI of libpbh: GPU Barnes-Hut distant ("regular") forces and
 * neighbour lists for the P3T scheme, on AMD Instinct MI355X (gfx950).
 *
 * Method: Arnold, Baumgardt & Wang (2021), "Accelerating NBODY6 with a
 * GPU-Enabled Particle-Particle Particle-Tree Scheme".
 *   - Section 2.1, eq. (fi) and the regular force F_R = (total) - F_I, with
 *     the changeover function K of eq. (duncan): every pair contributes
 *     m_j W(s) d/s^3 to F_R, W = 1 - K, d = x_j - x_i, s^2 = r^2 + eps^2.
 *   - Section 2.3: a constant neighbour radius; empty neighbour lists are
 *     legal. The list of i is { j != i : r_ij^2 < r_out^2 }.
 *   - Section 2.4: a Barnes-Hut tree with opening angle theta computes the
 *     regular force and fills the neighbour lists (REGF in the routine table
 *     of Appendix A); theta = 0 reduces to direct summation.
 *   - Section 2.2, eq. (kick): the leapfrog velocity kick with the regular
 *     force, used by pbh_kdk_graph and pbh_p3t.
 *
 * Conventions (all functions):
 *   - G = 1. r_out is the paper's r_cut; r_in its inner radius.
 *   - Pointers are DEVICE pointers unless marked "host". The caller owns
 *     every buffer it passes; the library owns its tree scratch.
 *   - pos is FP64 [n][3] row-major (x, y, z per particle), mass FP64 [n],
 *     acc FP64 [n][3], pot FP64 [n], all in the caller's particle order.
 *   - Neighbour lists are CSR: nbr_off int64 [n+1] (nbr_off[0] = 0),
 *     nbr_idx int32 [nbr_cap] holding caller-order indices. The order inside
 *     one list is unspecified (a list is a set) but deterministic.
 *   - The potential returned is the regular potential Phi_R, defined by
 *     dPhi_R/ds = W(s)/s^2 and Phi_R(s) = -1/s for s >= r_out (constant for
 *     s < r_in), so that F_R = -grad Phi_R exactly.
 *   - stream is a hipStream_t (NULL = the default stream). All work of a
 *     call is enqueued on it; calls return without waiting unless stated.
 *   - A context is not thread-safe: one call in flight per context.
 *   - Every call returns a status; on error pbh_last_error() gives a
 *     message. Nothing is printed.
 */
#ifndef PBH_H
#define PBH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbh_ctx pbh_ctx;
typedef void* pbh_stream_t; /* hipStream_t */

typedef enum {
    PBH_OK = 0,
    PBH_E_ARG = 1,           /* invalid argument (sizes, radii, theta, eps, NULL) */
    PBH_E_OOM = 2,           /* device allocation failed */
    PBH_E_HIP = 3,           /* a HIP runtime call failed */
    PBH_E_NONFINITE = 4,     /* NaN or Inf in pos or mass */
    PBH_E_NBR_OVERFLOW = 5,  /* nbr_cap too small; *nbr_total holds the size needed */
    PBH_E_STATE = 6,         /* force called without a matching build */
    PBH_E_INTERNAL = 7       /* a device-side capacity guard tripped */
} pbh_status;

typedef enum { PBH_FP64 = 0, PBH_MIXED = 1 } pbh_prec;

/*
 * Tuning parameters; 0 selects the default.
 *   leaf_size   n_leaf: a node with more particles is split (default 8)
 *   n_crit      particles per walk group, 1..64 (0: chosen per build, 32 below
 *               2^18 particles and 64 from there; one wave lane each)
 *   walk_tile   entries per LDS interaction tile of the walk: 64, 96 or 128
 *               (default 64); a tile is evaluated just before it would
 *               overflow, so larger tiles mean fewer evaluation rounds and
 *               fewer resident waves per compute unit
 *   lanes_per_particle  most wave lanes that share one particle of a small
 *               group, 1..64 (0: as many as fit, 64 / group size; 1: one
 *               lane per particle). The copies split the interaction tiles
 *               and their partial sums are merged in copy order.
 *   key_bits    Morton bits per axis D, 1..21 (default 21 for one cluster;
 *               batched builds use min(21, (63 - cluster bits) / 3))
 *   prec        PBH_MIXED (FP32 interactions, FP64 positions and sums) or
 *               PBH_FP64 (every interaction in FP64). Default PBH_MIXED.
 * Forces depend on leaf_size, n_crit and key_bits only through the tree's
 * approximation; walk_tile and lanes_per_particle change the order of the
 * FP32 tile sums only; neighbour lists depend on none of them.
 */
typedef struct {
    int32_t leaf_size;
    int32_t n_crit;
    int32_t walk_tile;
    int32_t lanes_per_particle;
    int32_t key_bits;
    int32_t prec;
} pbh_params;

/* Counters of the last build and force call (pbh_get_stats waits for the stream). */
typedef struct {
    int64_t n;            /* particles */
    int64_t n_clusters;
    int64_t n_nodes;
    int64_t n_leaves;
    int64_t n_groups;
    int64_t max_level;
    int64_t n_pn;         /* particle-node (multipole) interactions */
    int64_t n_pp_far;     /* particle-particle pairs outside r_out (W = 1) */
    int64_t n_pp_near;    /* pairs inside near leaves (changeover applied; self pairs counted) */
    int64_t nbr_total;    /* neighbour entries of the last force call */
    int64_t error_flags;  /* device-side guard bits; 0 when healthy (bit 5: pos or
                             mass changed since the build; bits 8-10: malformed
                             input of the last pbh_irregular call) */
    /* Phase durations of the last build / force call in milliseconds, from
       HIP events recorded on the call's stream; 0 unless timing is enabled
       (pbh_set_timing). walk = the tree-walk kernel alone. */
    double ms_build;
    double ms_walk;
    double ms_nbr;
    /* Lane slots of the walk's evaluation loops (64 per loop iteration of a
       wave) for multipole, far-pair and near-pair tiles. n_pn / lane_slots_pn
       etc. is the fraction of lanes doing useful work (idle lanes of groups
       smaller than a wave, copies beyond the tile's entries). */
    int64_t lane_slots_pn;
    int64_t lane_slots_far;
    int64_t lane_slots_near;
} pbh_stats;

/* Core quantities of pbh_core (Casertano & Hut 1985 estimator, see there). */
typedef struct {
    double center[3];   /* density centre x_d */
    double rho_core;    /* sum rho^2 / sum rho over the sample */
    double r_core;      /* sqrt(sum rho^2 |x - x_d|^2 / sum rho^2) */
    int64_t n_core;     /* particles with |x - x_d| < r_core (all n) */
    double r_half;      /* half-mass radius about x_d */
    double r_min;       /* 4 r_half / (n rho_core^(1/3)) */
    double dt_min;      /* 0.01 sqrt(eta / 0.02) sqrt(r_min^3) */
} pbh_core_info;

/* Create a context on HIP device `device`. params may be NULL (defaults). */
pbh_status pbh_create(int device, const pbh_params* params, pbh_ctx** out);
void pbh_destroy(pbh_ctx* ctx);
/* Replace the tuning parameters; takes effect at the next build. */
pbh_status pbh_set_params(pbh_ctx* ctx, const pbh_params* params);
pbh_status pbh_get_params(const pbh_ctx* ctx, pbh_params* out);

/*
 * Build the octree of one cluster (Section 2.4): bounding box and finiteness
 * check, Morton keys, stable radix sort, octree topology, FP64 monopole and
 * traceless quadrupole moments about each node's centre of mass, and walk
 * groups. n >= 1. pos/mass are read during the call's stream work only; the
 * library keeps its own sorted copy. Returns PBH_E_NONFINITE (after waiting
 * for the stream) if any coordinate or mass is NaN/Inf.
 */
pbh_status pbh_build(pbh_ctx* ctx, int64_t n, const double* pos, const double* mass,
                     pbh_stream_t stream);

/*
 * Regular force, regular potential and neighbour lists of the last build
 * (Section 2.1 eq. fi / F_R, eq. duncan; Section 2.3; Section 2.4; the
 * REGF contract of Appendix A: given the particles, return their regular
 * forces and neighbour lists).
 *   pos, mass    the arrays of the last pbh_build, unchanged since. Other
 *                pointers return PBH_E_STATE at once, as does a context
 *                without a successful single-cluster build. The walk also
 *                compares every particle's pos and mass with the build's
 *                sorted copy: a change in place since the build sets
 *                error_flags bit 5 (pbh_stats) and, when nbr_total is
 *                non-NULL (the call waits), returns PBH_E_STATE.
 *   r_in, r_out  changeover radii, 0 <= r_in <= r_out (r_out = 0: plain
 *                softened gravity and empty lists; r_in = r_out: step W)
 *   theta        opening angle >= 0 (0 = direct summation through the tree)
 *   eps          Plummer softening >= 0 (enters s, W and Phi_R, not the list)
 *   acc, pot     outputs [n][3], [n]
 *   nbr_off      [n+1] output, or NULL to skip the neighbour lists
 *   nbr_idx      [nbr_cap] output (may be NULL when nbr_cap = 0)
 *   nbr_total    host int64 out, or NULL. If non-NULL the call waits for the
 *                counts, stores the total, and returns PBH_E_NBR_OVERFLOW
 *                without filling nbr_idx when it exceeds nbr_cap (acc, pot
 *                and nbr_off are valid; resize and call again: the tree is
 *                reused). If NULL nothing waits; entries beyond nbr_cap are
 *                dropped and error_flags bit 0 is set in pbh_stats.
 */
pbh_status pbh_force(pbh_ctx* ctx, const double* pos, const double* mass, double r_in,
                     double r_out, double theta, double eps, double* acc, double* pot,
                     int64_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap, int64_t* nbr_total,
                     pbh_stream_t stream);

/*
 * pbh_force with a buffered neighbour radius (Section 2.3: R_cut = R_s +
 * R_buff; the run-parameter rule r_buff = 3 tau sigma): the lists hold every
 * j != i with r_ij^2 < (r_out + r_buff)^2, so they stay complete while the
 * particles move for a regular step. The changeover W still uses r_in and
 * r_out; nodes closer than r_out + r_buff to a walk group are opened to
 * particle pairs (W = 1 beyond r_out). r_buff finite and >= 0; r_buff = 0 is
 * pbh_force. The lists feed pbh_irregular unchanged (pairs beyond r_out add
 * nothing there).
 */
pbh_status pbh_force_buffered(pbh_ctx* ctx, const double* pos, const double* mass, double r_in,
                              double r_out, double r_buff, double theta, double eps, double* acc,
                              double* pot, int64_t* nbr_off, int32_t* nbr_idx, int64_t nbr_cap,
                              int64_t* nbr_total, pbh_stream_t stream);

/*
 * Ensemble of independent clusters built as one forest: cluster k holds
 * particles [offsets[k], offsets[k+1]) (host array, n_clusters + 1 entries,
 * offsets[0] = 0, each cluster non-empty). Keys carry the cluster id above
 * per-cluster Morton bits, so one sort orders every cluster; each cluster
 * gets its own root, bounding box and groups. 1 <= n_clusters <= 65536.
 */
pbh_status pbh_build_batched(pbh_ctx* ctx, int32_t n_clusters, const int64_t* offsets,
                             const double* pos, const double* mass, pbh_stream_t stream);

/*
 * Forces of every cluster of the last batched build in one persistent walk
 * launch. pos/mass are the arrays of that build (PBH_E_STATE otherwise, as
 * pbh_force). r_in/r_out are host arrays [n_clusters] (per-cluster
 * changeover radii); clusters never interact. Other arguments as pbh_force;
 * neighbour indices are global (caller-order) indices.
 */
pbh_status pbh_force_batched(pbh_ctx* ctx, const double* pos, const double* mass,
                             const double* r_in, const double* r_out, double theta, double eps,
                             double* acc, double* pot, int64_t* nbr_off, int32_t* nbr_idx,
                             int64_t nbr_cap, int64_t* nbr_total, pbh_stream_t stream);

/* pbh_force_batched with per-cluster buffers r_buff (host array [n_clusters],
   or NULL for none), as pbh_force_buffered. */
pbh_status pbh_force_batched_buffered(pbh_ctx* ctx, const double* pos, const double* mass,
                                      const double* r_in, const double* r_out,
                                      const double* r_buff, double theta, double eps,
                                      double* acc, double* pot, int64_t* nbr_off,
                                      int32_t* nbr_idx, int64_t nbr_cap, int64_t* nbr_total,
                                      pbh_stream_t stream);

/*
 * Irregular (neighbour) force, its time derivative and the irregular
 * potential from neighbour lists, in FP64 (Section 2.1, eq. fi, eq. fidot,
 * eq. duncan, eq. duncan2). With d = x_j - x_i, u = v_j - v_i,
 * s^2 = |d|^2 + eps^2, K = 1 - W and x = (s - r_in)/(r_out - r_in):
 *   acc_i  = sum_{j in list(i), j != i} m_j K(s) d / s^3
 *   jerk_i = sum m_j { K(s) [u / s^3 - 3 (d.u) d / s^5] + (dK/dt) d / s^3 },
 *            dK/dt = -140 x^3 (1-x)^3 (d.u) / (s (r_out - r_in)) on
 *            r_in <= s < r_out and 0 elsewhere (the term-by-term time
 *            derivative of eq. fi; eq. fidot as printed drops m_j and K from
 *            its second term, and eq. duncan2 has the opposite sign)
 *   pot_i  = sum m_j (-1/s - Phi_R(s)), so pot_i plus the regular potential
 *            of pbh_force is plain softened gravity.
 * Pairs with s >= r_out contribute nothing, so lists holding every j with
 * r_ij < r_out (the lists of pbh_force with the same r_out) give the whole
 * irregular force; lists of a larger radius give the same sums. A coincident
 * pair (s = 0) has no finite irregular force.
 *   n            particles, 1 <= n < 2^31
 *   pos, vel     [n][3] FP64 (vel may be NULL when jerk is NULL); mass [n]
 *   r_in, r_out  changeover radii as in pbh_force
 *   eps          Plummer softening >= 0
 *   nbr_off      [n+1] CSR offsets, nbr_idx [nbr_cap] caller-order indices
 *                (a list entry equal to i is skipped)
 *   targets      NULL: all n particles, outputs [n] in caller order; else a
 *                device int32 array of n_targets caller indices whose
 *                results go to outputs [n_targets] in that order (e.g. the
 *                active particles of a block time step); a non-NULL list
 *                with n_targets = 0 does nothing
 *   acc          output [.][3]; jerk [.][3] and pot [.] outputs or NULL
 *   check        1: wait for the stream and return PBH_E_ARG if a target,
 *                offset or list entry was out of range (it is skipped, never
 *                read); 0: do not wait, report such input in
 *                pbh_stats.error_flags bits 8 (list entry), 9 (offsets) and
 *                10 (target)
 * The call needs no build. When the context holds a build of n particles
 * and targets is NULL the particles are processed in its key order (faster;
 * the results are identical). The first such call after a build also finds
 * each particle's key position, which the context keeps until the next build.
 */
pbh_status pbh_irregular(pbh_ctx* ctx, int64_t n, const double* pos, const double* vel,
                         const double* mass, double r_in, double r_out, double eps,
                         const int64_t* nbr_off, const int32_t* nbr_idx, int64_t nbr_cap,
                         int64_t n_targets, const int32_t* targets,
                         double* acc, double* jerk, double* pot, int32_t check,
                         pbh_stream_t stream);

/*
 * pbh_irregular over the clusters of the last batched build: n and the
 * cluster ranges are the build's; r_in/r_out are host arrays [n_clusters]
 * and particle i takes the radii of its own cluster.
 */
pbh_status pbh_irregular_batched(pbh_ctx* ctx, const double* pos, const double* vel,
                                 const double* mass, const double* r_in, const double* r_out,
                                 double eps, const int64_t* nbr_off, const int32_t* nbr_idx,
                                 int64_t nbr_cap, int64_t n_targets, const int32_t* targets,
                                 double* acc, double* jerk, double* pot, int32_t check,
                                 pbh_stream_t stream);

/*
 * pbh_irregular for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, results and errors as pbh_irregular (the same kernels, so the
 * same sums bit for bit), except:
 *   - n <= PBH_NOALLOC_MAX_N (2^20); a larger n returns PBH_E_ARG.
 *   - The call allocates nothing. Its scratch (a flag word, and for the
 *     key-order route the ranks and 64-byte records of the n particles,
 *     68 MiB at the maximum n) is one static device array per GPU that the
 *     library holds from the first pbh_create on that GPU until the process
 *     ends. The flag word is cleared by a kernel at the start of every call,
 *     and the ranks are computed afresh by every call.
 *   - Every call on one GPU shares that array, from any context: calls that
 *     overlap in time on one GPU (other streams, other threads, other
 *     contexts) race and give undefined results. Order them on one stream.
 *   - With check = 0, malformed input is skipped (never dereferenced) but not
 *     reported in pbh_stats.error_flags; pass check = 1 to have it reported.
 * The context's build (if it holds one of these n particles) is used as by
 * pbh_irregular.
 */
#define PBH_NOALLOC_MAX_N 1048576
pbh_status pbh_irregular_noalloc(pbh_ctx* ctx, int64_t n, const double* pos, const double* vel,
                                 const double* mass, double r_in, double r_out, double eps,
                                 const int64_t* nbr_off, const int32_t* nbr_idx, int64_t nbr_cap,
                                 int64_t n_targets, const int32_t* targets, double* acc,
                                 double* jerk, double* pot, int32_t check, pbh_stream_t stream);

/*
 * Core quantities and regularisation parameters from the 6 nearest
 * neighbours of a particle sample (Section 3.2: a uniform sample of
 * min(N, sqrt(5000 N)) particles whose 6 nearest neighbours are searched
 * directly; Section 2.5: the regularisation parameters R_min and dT_min).
 * For each sampled particle i, with its 6 nearest neighbours among all n
 * particles (j != i, r^2 = (dx*dx + dy*dy) + dz*dz in FP64 without FMA, ties to
 * the lower index):
 *   rho_i = (sum of the masses of the 5 nearest) / ((4 pi / 3) r_6^3)
 * and the quantities of pbh_core_info over the sample (N_core and r_half over
 * all particles). The search runs through the octree of the last build and
 * returns the exact neighbours.
 *   pos, mass    the arrays of the last build (one cluster), n >= 7
 *   sample       device int32 [n_sample] distinct caller indices drawn by
 *                the caller (uniformly, without replacement), 1 <= n_sample <= n
 *   eta          accuracy parameter of the dT_min rule (the paper uses 0.02)
 *   rho          device FP64 [n_sample] out (per-sample densities), or NULL
 *   out          host struct, filled when the call returns (it waits)
 * PBH_E_ARG for a sample index outside [0, n); PBH_E_STATE without a
 * single-cluster build.
 */
pbh_status pbh_core(pbh_ctx* ctx, const double* pos, const double* mass, int64_t n_sample,
                    const int32_t* sample, double eta, double* rho, pbh_core_info* out,
                    pbh_stream_t stream);

/*
 * Hermite integration of the irregular force over one regular step dt_reg
 * (Section 2.2, step 3 of the integration algorithm), in place: pos and vel
 * [n][3] move under F_I only, each particle on its own block step dt_max / 2^k
 * with dt_max = dt_reg / 4 (eq. dtmax), predicted with eq. p3t-jpred-x and
 * p3t-jpred-dx (no regular force), corrected with the 4th-order Hermite
 * corrector, and given the next step by eq. dt (eta; a^(0) = F_I + fr). The
 * first step of every particle is eq. dt too, with the second and third time
 * derivatives of F_I computed from the lists along the motion under F_I
 * (Section 2.1, after eq. dt), and dt_max when the particle has no pair
 * inside r_out; steps at most double and stay commensurate with the block
 * time; all particles end at dt_reg.
 *   fr           [n][3] regular force for the step criterion, or NULL
 *   nbr_off/idx  lists that hold every pair inside r_out throughout the step
 *                (pbh_force_buffered with a large enough r_buff)
 *   stats        host int64[3] out or NULL: block steps, particle steps, the
 *                deepest level k
 * Block steps run in batches of 16 (one captured graph each); the host reads a
 * done flag once per batch while the next batch runs, and the call returns
 * after the stream has finished. The context keeps about 0.4 KB of device
 * state per particle (one bucket per level, 41 x 4 B, is most of it) until it
 * is destroyed; an allocation failure returns PBH_E_OOM.
 */
pbh_status pbh_hermite(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                       const double* fr, double r_in, double r_out, double eps,
                       const int64_t* nbr_off, const int32_t* nbr_idx, int64_t nbr_cap,
                       double dt_reg, double eta, int64_t* stats, pbh_stream_t stream);

/*
 * The P3T loop (Section 2.2, the integration algorithm): regular force and
 * lists of radius r_out + r_buff at the start (tree walk with theta, the
 * context's precision); then per step: v += dt_reg/2 F_R (eq. kick); Hermite
 * integration of F_I over dt_reg (pbh_hermite); regular force and lists
 * again; v += dt_reg/2 F_R. pos, vel updated in place. energy_out: device
 * FP64 [steps+1] or NULL: sum m v^2/2 + sum m (Phi_R + Phi_I)/2 (plain
 * softened gravity) before the first step and after each. stats as in
 * pbh_hermite, summed over the steps. The library keeps its own neighbour
 * buffer (grown as needed).
 */
pbh_status pbh_p3t(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                   double r_in, double r_out, double r_buff, double theta, double eps,
                   double dt_reg, double eta, int32_t steps, double* energy_out, int64_t* stats,
                   pbh_stream_t stream);

/*
 * Kick-drift-kick leapfrog under the regular force (Section 2.2, eq. kick and
 * the loop that follows it), with a full tree rebuild every step:
 *   a = F_R(x); repeat steps times { v += dt/2 a; x += dt v; rebuild;
 *   a = F_R(x); v += dt/2 a; E = sum m v^2/2 + sum m Phi_R/2 }.
 * One step is captured once into a hipGraph and replayed `steps` times.
 * pos/vel [n][3] are updated in place; energy_out is a device array
 * [steps+1] (energy before the first step, then after each). n is fixed at
 * the first call for this context; later calls with the same n reuse the graph.
 */
pbh_status pbh_kdk_graph(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                         double dt, int32_t steps, double r_in, double r_out, double theta,
                         double eps, double* energy_out, pbh_stream_t stream);

/* Same step sequence launched eagerly (no graph), for replay checks. */
pbh_status pbh_kdk_eager(pbh_ctx* ctx, int64_t n, double* pos, double* vel, const double* mass,
                         double dt, int32_t steps, double r_in, double r_out, double theta,
                         double eps, double* energy_out, pbh_stream_t stream);

/* Record HIP events around the build, walk and neighbour phases of later
   eager calls (enable = 1) or stop (0). Costs a few microseconds per call. */
pbh_status pbh_set_timing(pbh_ctx* ctx, int32_t enable);

/* Waits for the stream of the last call, then fills *out. */
pbh_status pbh_get_stats(pbh_ctx* ctx, pbh_stats* out);

/*
 * Rate of the device cycle counter (clock64) during the last tree walk, in MHz:
 * a measurement beside the roofline figures, not a step of the paper's method.
 * Every workgroup of the walk records the cycle-counter and steady-clock
 * counts between its start and its end; *mhz is the sum of the cycles over
 * the sum of the ticks at the device's steady-clock rate. Waits for the
 * stream. PBH_E_STATE before any walk (or after buffers were reallocated),
 * PBH_E_ARG for null arguments.
 */
pbh_status pbh_walk_clock(pbh_ctx* ctx, double* mhz);

/*
 * Debug export of the last build (waits for the stream). Host buffers:
 *   order [n]          sorted position -> caller index (int32)
 *   keys  [n]          sorted keys (uint64)
 *   nodes_i [cap][4]   begin, count, nchild, level (int64) in pre-order
 *   nodes_d [cap][16]  M, com[3], q[6] (xx,yy,zz,xy,xz,yz), lo[3], hi[3]
 * Any pointer may be NULL. Returns PBH_E_ARG if cap < node count (which is
 * written to *n_nodes).
 */
pbh_status pbh_debug_tree(pbh_ctx* ctx, int32_t* order, uint64_t* keys, int64_t cap,
                          int64_t* nodes_i, double* nodes_d, int64_t* n_nodes);

/*
 * Debug export of the walk groups of the last build (waits for the stream):
 * first sorted particle and particle count of each group, in particle order,
 * and its tight box (lo xyz, hi xyz). Host buffers of cap entries, or NULL.
 * The group count is written to *n_groups; PBH_E_ARG if cap is too small.
 */
pbh_status pbh_debug_groups(pbh_ctx* ctx, int64_t cap, int32_t* begin, int32_t* count,
                            double* box /* [cap][6] */, int64_t* n_groups);

/*
 * Debug export of the persistent launches of the last walk and neighbour
 * count: for each workgroup, the number of groups it processed and its
 * run time in ticks of the 100 MHz device wall clock. Host buffers of
 * [cap][2] uint64; the workgroup counts go to *n_walk and *n_nbr.
 */
pbh_status pbh_debug_wave_log(pbh_ctx* ctx, uint64_t* walk, uint64_t* nbr, int64_t cap,
                              int64_t* n_walk, int64_t* n_nbr);

/*
 * Debug export of the first block step (in ticks of dt_max / 2^40) that the
 * last pbh_hermite call (or the last regular step of pbh_p3t) gave each
 * particle, caller order. Host buffer of cap entries, or NULL; the particle
 * count goes to *n_out. PBH_E_STATE before any integration.
 */
pbh_status pbh_debug_herm_first_steps(pbh_ctx* ctx, int64_t cap, int64_t* ticks, int64_t* n_out);

/*
 * Calibration kernel for hardware instruction counters: `blocks` waves, each
 * issuing exactly 32 * iters + 32 VALU instructions (32 * iters of them FP32
 * FMAs). out: device float [blocks], normally left unwritten.
 */
pbh_status pbh_debug_valu_probe(pbh_ctx* ctx, int64_t blocks, int32_t iters, float* out,
                                pbh_stream_t stream);

/*
 * Debug evaluation of the natural logarithm that the irregular potential uses
 * for Phi_R (the atanh-series form of the irregular-force kernels, not the
 * library's): y[k] = ln x[k] for k < n. x: device double [n], each positive
 * and normal; y: device double [n]. Enqueued on `stream`, nothing allocated.
 */
pbh_status pbh_debug_series_log(pbh_ctx* ctx, int64_t n, const double* x, double* y,
                                pbh_stream_t stream);

const char* pbh_last_error(const pbh_ctx* ctx);
const char* pbh_status_string(pbh_status s);

#ifdef __cplusplus
}
#endif

#endif /* PBH_H */
