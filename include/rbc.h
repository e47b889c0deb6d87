/*
 * rbc.h -- C ABI of the MI355X (gfx950) short-range force / time-step library
 * for the two-component CGMD red-cell membrane model (OpenRBC, Tang et al.).
 *
 * What the library computes (paper sections cited by name; the paper gives
 * no potential, so the model constants are parameters):
 *  - rbc_update_cells: the adaptive "lattice-free" cell list of the Spatial
 *    Searching Algorithm section -- Voronoi cells of k-means centroids over
 *    the lipid particles, kept current by an online expectation-maximisation
 *    update (nearest-centroid assignment, centroid move), centroids ordered
 *    along a Morton curve and particles reordered by owning cell (the
 *    two-level reordering), plus the cell-pair and per-particle neighbour
 *    lists derived from them.  Protein beads join the lipids' cells, or, for
 *    a detached cytoskeleton (params.protein_cells), a second set of cells
 *    built the same way over the protein beads alone (Force Evaluation
 *    section); cell pairs then also span the two sets.
 *  - rbc_forces: pairwise forces and torques between lipids, lipids and
 *    proteins and between proteins found through those cells, plus the bond
 *    list of physically linked proteins (Force Evaluation section).
 *  - rbc_step: the time-stepping loop of the Software Overview section: force
 *    and torque on every particle drive position and orientation updates
 *    (velocity Verlet with a free linear-rotor drift for lipid orientations).
 *
 * Conventions.
 *  - Array pointers marked [device] are HIP device pointers (for example
 *    torch CUDA tensors' data_ptr()).  n x 3 arrays are C-contiguous row-major
 *    FP64.  All device work is enqueued on the library's own stream, which is
 *    ordered after the caller's stream (passed at create) on entry and before
 *    it on return, so callers may treat every call as stream-ordered on their
 *    stream.  Calls marked (sync) also wait for completion.
 *  - Ownership: the caller owns every buffer it passes.  Inputs are copied
 *    into library-owned, cell-sorted storage before the call returns
 *    (stream-ordered); outputs are written in the caller's particle order.
 *  - Errors: every call returns rbc_status.  Argument errors return before
 *    any work is enqueued.  Device-side errors (capacity overflow, non-finite
 *    state, a missed neighbour-list rebuild) are reported by the call that
 *    observes them.  rbc_last_error() gives text.  A handle is not
 *    thread-safe.
 *  - Particle types: 0 = lipid, 1 = spectrin bead, 2 = junction.  Only lipids
 *    carry an orientation (unit vector) and angular velocity; proteins'
 *    orientation and angular velocity entries are ignored and returned zero.
 */
#ifndef RBC_H
#define RBC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbc_ctx *rbc_handle;

typedef enum {
    RBC_OK = 0,
    RBC_ERR_INVALID_ARG = 1,   /* bad pointer, size or parameter; nothing was enqueued */
    RBC_ERR_OUT_OF_MEMORY = 2, /* device allocation failed */
    RBC_ERR_HIP = 3,           /* HIP runtime error (no device, launch failure, ...) */
    RBC_ERR_NOT_READY = 4,     /* no system loaded / slot not live */
    RBC_ERR_CAPACITY = 5,      /* a neighbour or cell-pair list overflowed, or no slot / budget left */
    RBC_ERR_NONFINITE = 6,     /* NaN or Inf in the state */
    RBC_ERR_UNSUPPORTED = 7,   /* parameter combination the kernels do not implement */
    RBC_ERR_SKIN = 8           /* a particle moved beyond the skin before the lists were rebuilt */
} rbc_status;

typedef enum { RBC_FP64 = 0, RBC_MIXED = 1 } rbc_precision;

/* Model and cell-list parameters (sigma = epsilon = m = 1 units).
 * rc[t][u]: pair cutoff for types t,u; rc[0][0] is the lipid potential's r_c.
 * The neighbour set is every pair whose min-image FP64 squared distance,
 * summed as (dx*dx + dy*dy) + dz*dz with no fused multiply-add, is strictly
 * below fl(rc*rc).  zeta must be a positive integer (<= 16). */
typedef struct {
    double rc[3][3];
    double eps, zeta, mu, sin_theta0, r_min;   /* lipid orientation-dependent pair law */
    double wca_eps, wca_sigma;                  /* WCA for pairs involving proteins */
    double k_bond;                              /* harmonic bonds; rest length per bond */
    double mass[3];                             /* per type */
    double inertia;                             /* lipid rotational inertia */
    int32_t cell_target;                        /* mean lipids per Voronoi cell (k = ceil(N_L / m)) */
    int32_t update_every;                       /* online-EM cell update period in steps */
    double skin;                                /* displacement bound between updates (sigma) */
    int32_t lloyd_iters;                        /* k-means iterations when cells are first built */
    int32_t precision;                          /* rbc_precision: FP32 pair arithmetic or FP64 */
    int32_t protein_cells;                      /* 0: protein beads join the lipids' Voronoi cells (a
                                                   cytoskeleton attached to the bilayer); 1: they get a
                                                   separate set of cells, ceil(N_P / cell_target) of
                                                   them (a detached cytoskeleton) -- Force Evaluation
                                                   section */
    /* Harmonic volume constraint (the Validation and Benchmark section's whole-cell fluctuation run
     * keeps the cell's surface-to-volume ratio with one; its form is a reading):
     * U_V = vol_k/2 (V - V0)^2 / V0 with V = lipid_area/3 sum over lipids of
     * (x_i - xbar).n_i, xbar the lipid centroid (divergence theorem; lipid
     * orientations are the outward normals).  Open boundaries only. */
    double vol_k;                               /* 0: off */
    double vol_target;                          /* V0; 0: the V of the loaded state */
    double lipid_area;                          /* membrane area per lipid */
    /* Langevin thermostat (a reading; the paper names none): after each step's
     * closing half-kick, v <- c v + sqrt((1 - c^2) kT / m) xi with c = exp(-gamma dt),
     * and for lipids w <- c_r w + sqrt((1 - c_r^2) kT / I) (xi' - (xi'.n) n).
     * xi, xi': unit-variance uniform deviates from Philox4x32-10 (Salmon et al.,
     * SC'11) with counter (particle id, step low and high words, 0 or 1) and key
     * (seed low and high words); steps count from 1 after loading. */
    double kT;
    double gamma;                               /* translational friction rate; 0: none */
    double gamma_rot;                           /* lipid rotational friction rate; 0: none */
    uint64_t seed;
    /* Velocity quenching, the relaxation the Initial structure generation section
     * applies to a generated structure (the rule is a reading): after each closing
     * half-kick a particle keeps only the part of its velocity along its force,
     * v <- max(v.F, 0) F / |F|^2, and a lipid likewise the part of its angular
     * velocity along its torque; before each drift |v| dt and |w| dt are capped at
     * quench_max.  Excludes the thermostat. */
    double quench_max;                          /* sigma per step (radians for rotations) */
    int32_t quench;                             /* 1: quench instead of free dynamics */
    /* Pruned lists.  The neighbour lists are built with the full skin (radius rc + 2
     * skin) every update_every steps or when a particle could move more than the
     * skin; between builds the step kernel walks pruned copies that keep only the
     * partners within rc + 2 inner_skin at the moment of pruning, refreshed from the
     * full lists whenever a particle could move more than inner_skin since the last
     * prune.  A value outside (0, skin) prunes only at the builds (pruned lists =
     * full lists).  The neighbour set is unchanged either way. */
    double inner_skin;
} rbc_params;

/* ---- single-system context (an ensemble with one slot) ---- */

/* Create a context on the current HIP device.  hip_stream: the caller's
 * hipStream_t (0 = the null stream).  No device memory is sized until a system
 * is set. */
rbc_status rbc_create(const rbc_params *params, void *hip_stream, rbc_handle *out);

/* Load a system (sync).  [device] x, nrm, v, w: n x 3; type: n; bonds: nbond x 2
 * particle ids; r0: nbond rest lengths.  [host] box[3] lengths and periodic[3]
 * flags (1 = periodic axis; box ignored on open axes).  Periodic lengths must
 * exceed twice the largest cutoff plus skin.  0 <= n <= 2^29; n = 0 clears the
 * context.
 * Builds the initial Voronoi cells (params.lloyd_iters k-means iterations). */
rbc_status rbc_set_system(rbc_handle h, int64_t n, const double *x, const double *nrm,
                          const int32_t *type, const double *v, const double *w,
                          int64_t nbond, const int32_t *bonds, const double *r0,
                          const double *box, const int32_t *periodic);

/* Rebuild the cells now.  lloyd_iters > 0: re-seed from the lipids (and the
 * protein beads, for a separate protein cell set) and run that
 * many k-means iterations first; 0: one online-EM update (assign, move
 * centroids, Morton reorder, particle reorder, cell and neighbour lists). */
rbc_status rbc_update_cells(rbc_handle h, int32_t lloyd_iters);

/* Forces and torques at the current positions.  [device] F, T: n x 3 outputs in
 * caller order (either may be NULL).  [device, nullable] energy: 2 doubles,
 * potential energy U and scalar virial W = sum over pairs and bonds of
 * r_ij . F_ij. */
rbc_status rbc_forces(rbc_handle h, double *F, double *T, double *energy);

/* Advance nsteps of NVE velocity Verlet with time step dt (sync at the end).
 * Cells are updated every update_every steps and earlier when a particle
 * could move more than the skin. */
rbc_status rbc_step(rbc_handle h, int64_t nsteps, double dt);

/* Copy the state out in caller order.  [device] n x 3 each; any may be NULL. */
rbc_status rbc_get_state(rbc_handle h, double *x, double *nrm, double *v, double *w);

/* The current neighbour set as sorted pairs (i < j) of caller ids (sync).
 * [host] ij: cap x 2.  *npairs receives the full count even when it exceeds cap. */
rbc_status rbc_get_pairs(rbc_handle h, int64_t cap, int32_t *ij, int64_t *npairs);

/* rbc_get_pairs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pairs, sorted the same way, but staged in a static device array of 32 MiB that
 * each GPU the library runs on holds until the process ends, instead of a buffer the
 * library allocates.  It calls no hipMalloc, hipFree or other allocating routine.
 * Limits: at most (32 MiB - 256 B) / 8 = 4,194,272 pairs; a larger set returns
 * RBC_ERR_CAPACITY with *npairs unset.  [host] ij: cap x 2; the sorted pairs are
 * written only when cap >= the count (otherwise nothing is written and *npairs
 * receives the count).  Every call on one GPU shares that GPU's staging array, which
 * keeps the last call's contents: calls that overlap on one GPU (from several
 * threads or contexts) race and must be serialised by the caller. (sync) */
rbc_status rbc_get_pairs_noalloc(rbc_handle h, int64_t cap, int32_t *ij, int64_t *npairs);

/* Energies of the current state (sync).  [host] out[7]: U (with U_V when the
 * volume constraint is on), W (pairs and bonds), kinetic energy (translational +
 * lipid rotational), total E = KE + U, |sum F|, |sum (r x F + tau)|, and the
 * volume V of the lipid surface (as defined for the volume constraint). */
rbc_status rbc_energy(rbc_handle h, double *out);

/* Counters (sync).  [host] out[11]: steps done, neighbour-list builds (all
 * kinds), list-only rebuilds (the skin ran out between cell updates), cells k,
 * max neighbour-list rows, max cell-pair row, particles n, lipids, lipid cells
 * (cells [0, out[8]) hold lipids; with protein_cells set, cells [out[8], k)
 * hold the protein beads; otherwise out[8] == k), Voronoi cell updates
 * (the initial build included; every params.update_every steps, each also
 * rebuilding the lists), and prunes of the lists between builds. */
rbc_status rbc_stats(rbc_handle h, int64_t *out);

/* Cell structure for inspection (sync).  [host] owner: n ints, the cell of
 * each particle in caller order; seeds: k x 3 cell centroids in cell order;
 * either may be NULL. */
rbc_status rbc_get_cells(rbc_handle h, int32_t *owner, double *seeds);

/* Average duration in milliseconds of the pair-force kernel launches since the
 * last call (measured with HIP events on the library stream around each launch
 * when timing is enabled), and the number of launches timed. */
rbc_status rbc_force_timing(rbc_handle h, int32_t enable, double *avg_ms, int64_t *launches);

/* Average duration in milliseconds of the list-build kernel launches (one per list
 * build or cell update, building every rebuilding system's lists and pruned lists)
 * timed while force timing was enabled, since the last call, and their number
 * (sync).  Timing keeps at most 64 launches between harvests, which every 256 timed
 * steps and every call of this function or rbc_force_timing make. */
rbc_status rbc_build_timing(rbc_handle h, double *avg_ms, int64_t *launches);

/* Per-step timing of the last rbc_step / rbc_ensemble_step call made while step
 * timing was on: [host] ms[q] (at most cap) the GPU interval of step q, from the end
 * of the previous step's launches (for q = 0, the start of the call) to the end of
 * its own, cell updates, list builds and prunes of that step included; *count the
 * number of steps; *gap_ms (nullable) the time from the end of the previous timed
 * call to the start of the last one (-1 when there is none).  enable turns the
 * timing (an event per step) on or off for later calls. */
rbc_status rbc_step_times(rbc_handle h, int32_t enable, int64_t cap, double *ms, int64_t *count, double *gap_ms);

/* Host time per step of the last rbc_step / rbc_ensemble_step call: [host] *host_us
 * the microseconds per step the calling thread spent outside waits for the device
 * (step decisions and kernel launches, cell-update launches included), *wait_us the
 * microseconds per step it waited for the drift statistics of earlier steps.  Either
 * pointer may be NULL; both read -1 before the first call.  No device work. */
rbc_status rbc_host_times(rbc_handle h, double *host_us, double *wait_us);

/* Replay the step's fixed launch sequence (the force kernel with its fused drift
 * and the drift statistics) as a HIP graph captured once per system table and time
 * step (enable = 1), or launch every kernel directly (0).  Cell updates always
 * launch directly, with grids covering only the systems that rebuild.  Results are
 * identical either way.  Default: off (the step is two launches, and a graph launch
 * costs the host more than the two direct ones).  Graphs are not used while force
 * timing is enabled.  Synchronises the library stream. */
rbc_status rbc_set_graphs(rbc_handle h, int32_t enable);

/* Internal cell-list arrays of the single system, for inspection and tests (sync).
 * which: 0 owner (n, slot order), 1 cell start (k+1), 2 cell count (k), 3 cell-pair
 * row start (k+1), 4 cell-pair entries (row start[k]), 5 seed-grid start (cells+1),
 * 6 seeds in grid order (k), 7 centroids with radius (k x 4 doubles), 8 list rows per
 * 64-particle chunk, 9 staged count per 256-particle block, 10 caller id per slot (n),
 * 11 segmented-scan tile sums, 12 pruned stage count per 256-particle block (-1: the
 * block keeps its full 32-bit lists), 13 pruned-list rows per 64-particle chunk.
 * Integer arrays are int32.  [host] out receives at most cap bytes; *bytes the full size. */
rbc_status rbc_debug_array(rbc_handle h, int32_t which, int64_t cap, void *out, int64_t *bytes);

rbc_status rbc_sync(rbc_handle h);
rbc_status rbc_destroy(rbc_handle h);
const char *rbc_status_string(rbc_status s);
const char *rbc_last_error(rbc_handle h);

/* ---- ensemble: continuous batching of independent systems ----
 * Systems live in slots; every call to rbc_ensemble_step advances all live
 * slots together with batched launches.  A system's trajectory does not depend
 * on which other systems share the batch. */

/* max_slots <= 256; hbm_budget_bytes: admission limit on device memory (0 = no limit). */
rbc_status rbc_ensemble_create(const rbc_params *params, void *hip_stream, int32_t max_slots,
                               int64_t hbm_budget_bytes, rbc_handle *out);
/* Device bytes a system of n particles (nlip lipids) and nbond bonds would take. */
rbc_status rbc_ensemble_footprint(rbc_handle h, int64_t n, int64_t nlip, int64_t nbond, int64_t *bytes);
/* Admit a system (arrays as rbc_set_system).  Returns RBC_ERR_CAPACITY when no
 * slot is free or the footprint exceeds the remaining budget; *slot receives
 * the slot index. */
rbc_status rbc_ensemble_admit(rbc_handle h, int64_t n, const double *x, const double *nrm,
                              const int32_t *type, const double *v, const double *w,
                              int64_t nbond, const int32_t *bonds, const double *r0,
                              const double *box, const int32_t *periodic, int32_t *slot);
/* Admission in two phases, for callers that admit several systems at once.
 * rbc_ensemble_stage validates, allocates and uploads a system exactly as
 * rbc_ensemble_admit does (same arguments, same errors, *slot receives the slot;
 * the input arrays may be released on return) but leaves its cell build pending.
 * rbc_ensemble_commit then builds the cells of every pending slot in one set of
 * launches: the seeding, Lloyd iterations and reordering of the Spatial
 * Searching Algorithm section, then the cell pairs and lists of the Force Evaluation
 * section.  Each system's result equals that of rbc_ensemble_admit.  A slot whose
 * build fails (capacity, non-finite input) is released and its index written to
 * failed[0..min(*nfailed, cap)); rbc_last_error holds the first failure's message,
 * and commit still returns RBC_OK.  While a slot is pending, the calls that need
 * built cells (rbc_ensemble_step, rbc_ensemble_energy, rbc_update_cells, rbc_forces,
 * rbc_get_pairs, rbc_get_cells) return RBC_ERR_NOT_READY. */
rbc_status rbc_ensemble_stage(rbc_handle h, int64_t n, const double *x, const double *nrm,
                              const int32_t *type, const double *v, const double *w,
                              int64_t nbond, const int32_t *bonds, const double *r0,
                              const double *box, const int32_t *periodic, int32_t *slot);
rbc_status rbc_ensemble_commit(rbc_handle h, int64_t cap, int32_t *failed, int64_t *nfailed);
/* Advance every live slot by nsteps (sync at the end). */
rbc_status rbc_ensemble_step(rbc_handle h, int64_t nsteps, double dt);
/* State of one slot in its caller order ([device] n x 3 each, any may be NULL). */
rbc_status rbc_ensemble_get_state(rbc_handle h, int32_t slot, double *x, double *nrm, double *v, double *w);
/* Energies of one slot ([host] out[7] as rbc_energy). */
rbc_status rbc_ensemble_energy(rbc_handle h, int32_t slot, double *out);
/* Free a slot and its memory. */
rbc_status rbc_ensemble_retire(rbc_handle h, int32_t slot);
/* Slots frozen by an error (ensemble contexts).  When a slot's lists overflow
 * (RBC_ERR_CAPACITY), its state turns non-finite (RBC_ERR_NONFINITE) or a particle
 * outruns the skin (RBC_ERR_SKIN) during rbc_ensemble_step, that call returns the
 * first such status, every other live slot has still advanced nsteps, and the failed
 * slot is frozen: it keeps its slot and memory but takes no further part in any
 * launch, and its state and energy calls return its status, until it is retired.  A
 * retry cannot help these errors (an overflow is fixed by the positions, which the
 * steps with truncated lists already changed), so the library isolates the slot
 * instead.  [host] slots, status: the failed slots and their statuses, at most cap;
 * *count receives the full number. */
rbc_status rbc_ensemble_failed(rbc_handle h, int64_t cap, int32_t *slots, int32_t *status, int64_t *count);
/* [host] out[4]: live slots, device bytes in use, budget, steps done by the ensemble. */
rbc_status rbc_ensemble_info(rbc_handle h, int64_t *out);

#ifdef __cplusplus
}
#endif
#endif
