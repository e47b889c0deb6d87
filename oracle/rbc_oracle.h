/*
 * Plain FP64 CPU oracle for the short-range force / time-step path of the
 * two-component CGMD red-cell membrane model (OpenRBC, Tang et al.).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two meet only through the
 * seeded input generator.
 *
 * Everything here is the plain definition, written for a reader to check by
 * eye: brute-force or uniform-grid pair enumeration with one exact FP64
 * distance test, per-pair potentials, per-particle sums, a textbook
 * velocity-Verlet / linear-rotor step, and the deterministic Voronoi
 * (k-means) reference steps used to unit-test the GPU cell build.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math): every FP64
 * operation is rounded separately, which the bit-exact neighbour test needs.
 *
 * Pins (what fixes each function besides itself; see tests/test_oracle_*.py):
 *   orc_pair_lipid   central finite differences of U for F and torque; closed
 *                    values at r_min (parallel -eps, antiparallel (2mu-1)eps,
 *                    stacked (mu-1)eps); zero at and beyond r_c; continuity at
 *                    r_min and r_c; swap, rotation and n -> -n invariance;
 *                    per-pair momentum and angular-momentum identities.
 *                    The potential's form and constants are a reading: the
 *                    paper cites its membrane model without stating it, so
 *                    they are parity unpinned against the paper itself.
 *   orc_pair_wca     textbook closed form; zero value and force at 2^(1/6) sigma.
 *   orc_bond         harmonic closed form; dimer period 2 pi / sqrt(2k/m).
 *   orc_pairs_*      brute force O(N^2) == uniform grid, bit for bit; the flat
 *                    patch has exactly 18 lipid neighbours per lipid.
 *   orc_forces*      FD of the total energy; sum F = 0; sum(r x F + tau) = 0
 *                    on open boundaries; energy == sum of pair energies.
 *   orc_assign       brute-force argmin (the definition itself).
 *   orc_seed_update  Lloyd objective non-increasing; centroid of a cell.
 *   orc_morton       hand-computed keys for known points.
 *   orc_vv_run       energy error falls ~4x when dt halves; time reversal;
 *                    free rotor; harmonic dimer period.
 *   orc_philox4x32_10  the generator's published known-answer vectors.
 *   orc_volume       sphere and Evans-Fung cell volumes (closed form and
 *                    quadrature); translation and rotation invariance.
 *   orc_volume_forces  finite differences of U_V in x and n; sum F = 0 and
 *                    sum(r x F + tau) = 0.
 *   orc_langevin_step  deviates' mean and variance; equipartition of free
 *                    particles and free rotors (<m v^2> = 3 kT, <I w^2> = 2 kT);
 *                    the exact decay of the mean velocity.
 *   orc_quench_*     hand-computed projections and caps; a harmonic dimer and
 *                    a stretched chain relax to their minima; the energy of an
 *                    overlapping structure falls monotonically.
 */
#ifndef RBC_ORACLE_H
#define RBC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double box[3];
    int32_t periodic[3];
    double rc[3][3];          /* cutoff per type pair; rc[0][0] is the lipid r_c */
    double eps, zeta, mu, sin_theta0, r_min;
    double wca_eps, wca_sigma;
    double k_bond;
    double mass[3];
    double inertia;
} orc_params;

/* Min-image difference d = x_i - x_j and the exact FP64 squared distance. */
double orc_dist2(const orc_params *p, const double *xi, const double *xj, double *d);

/* Lipid-lipid orientation-dependent pair.  d = x_i - x_j.  Returns U; writes the
 * force on i (force on j is -Fi) and the torques on i and j. */
double orc_pair_lipid(const orc_params *p, const double *d, const double *ni, const double *nj,
                      double *Fi, double *ti, double *tj);
/* WCA pair for any pair involving a protein bead.  Returns U; writes force on i. */
double orc_pair_wca(const orc_params *p, const double *d, double *Fi);
/* Harmonic bond.  Returns U; writes force on i. */
double orc_bond(const orc_params *p, const double *d, double r0, double *Fi);

/* Neighbour set: all pairs (i<j) with dist2 < fl(rc*rc); written as sorted (i,j).
 * Returns the pair count (writes at most cap pairs). */
int64_t orc_pairs_brute(const orc_params *p, int64_t n, const double *x, const int32_t *type,
                        int64_t cap, int32_t *ij);
int64_t orc_pairs_grid(const orc_params *p, int64_t n, const double *x, const int32_t *type,
                       int64_t cap, int32_t *ij);

/* Forces, torques, U and the scalar virial W over all pairs of the neighbour
 * set and all bonds.  energy[0] = U, energy[1] = W.  nthreads <= 0: OpenMP default. */
int orc_forces(const orc_params *p, int64_t n, const double *x, const double *nrm,
               const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
               double *F, double *T, double *energy, int nthreads);
/* Forces on the listed particles only, by brute force over every partner. */
int orc_forces_subset(const orc_params *p, int64_t n, const double *x, const double *nrm,
                      const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
                      int64_t nsub, const int64_t *idx, double *F, double *T, int nthreads);

/* Voronoi reference steps. */
void orc_assign(const orc_params *p, int64_t n, const double *x, int64_t k, const double *seeds,
                int32_t *owner);
void orc_seed_update(const orc_params *p, int64_t n, const double *x, const int32_t *type,
                     const int32_t *owner, int64_t k, double *seeds);
void orc_morton(const orc_params *p, int64_t k, const double *seeds, uint64_t *keys);
void orc_cell_bounds(const orc_params *p, int64_t n, const double *x, const int32_t *owner,
                     int64_t k, const double *seeds, double *R);
int64_t orc_cell_pairs(const orc_params *p, int64_t k, const double *seeds, const double *R,
                       double rs, double skin, int64_t cap, int32_t *ab);

/* NVE velocity Verlet with the free linear-rotor drift.  energies (nsteps+1) x 3:
 * KE, U, KE+U at every step (entry 0 = initial).  State arrays updated in place. */
int orc_vv_run(const orc_params *p, int64_t n, double *x, double *v, double *nrm, double *w,
               const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
               double dt, int64_t nsteps, double *energies, int nthreads);

/* ---- Beyond the conservative model: a harmonic volume constraint (the
 * whole-cell fluctuation run of the Validation and Benchmark section keeps the cell's
 * surface-to-volume ratio with one) and a Langevin thermostat.  The paper
 * states neither form; these are readings. */
typedef struct {
    double vol_k;        /* k_V of U_V = k_V/2 (V - V0)^2 / V0; 0 = no volume term */
    double vol_target;   /* V0 */
    double lipid_area;   /* a_L, membrane area per lipid */
    double kT;           /* thermostat temperature */
    double gamma;        /* translational friction rate; 0 = none */
    double gamma_rot;    /* lipid rotational friction rate; 0 = none */
    uint64_t seed;       /* Philox key */
    double quench_max;   /* velocity quenching: largest move per step (sigma, and radians for
                            a lipid's rotation) */
    int32_t quench;      /* 1: velocity quenching instead of free dynamics */
    int32_t pad;
} orc_ext;

/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): counter ctr, key key. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Enclosed volume from the lipids by the divergence theorem: each lipid stands for
 * a membrane patch of area a_L with outward normal n_i, so
 * V = (a_L / 3) sum_i (x_i - xbar) . n_i with xbar the lipid centroid. */
double orc_volume(const orc_ext *e, int64_t n, const double *x, const double *nrm, const int32_t *type);

/* Adds -dU_V/dx_i to F and n_i x (-dU_V/dn_i) to T (lipids only); returns U_V. */
double orc_volume_forces(const orc_ext *e, int64_t n, const double *x, const double *nrm,
                         const int32_t *type, double *F, double *T);

/* orc_forces plus the volume term (energy[0] includes U_V; energy[1], the pair and
 * bond virial, does not). */
int orc_forces_ext(const orc_params *p, const orc_ext *e, int64_t n, const double *x, const double *nrm,
                   const int32_t *type, int64_t nbond, const int32_t *bonds, const double *r0,
                   double *F, double *T, double *energy, int nthreads);

/* The thermostat's exact Ornstein-Uhlenbeck velocity update for step number `step`:
 * v <- c v + sqrt((1 - c^2) kT / m) xi with c = exp(-gamma dt); for lipids also
 * w <- c_r w + sqrt((1 - c_r^2) kT / I) (xi' - (xi'.n) n).  xi, xi' hold unit-variance
 * uniform deviates from Philox4x32-10 with counter (particle id, step low word,
 * step high word, 0 or 1) and key (seed low word, seed high word). */
void orc_langevin_step(const orc_params *p, const orc_ext *e, int64_t n, const int32_t *type,
                       const double *nrm, double dt, uint64_t step, double *v, double *w);

/* Velocity quenching (Initial structure generation section: the generated
 * structure is relaxed by velocity quenching; the rule is a reading): after the
 * closing half-kick each particle keeps only the part of its velocity along its
 * force, v <- max(v.F, 0) F / |F|^2 (v <- 0 where F = 0), and each lipid the
 * part of its angular velocity along its torque.  The opening half-kick's
 * velocity is then capped so that one drift moves a particle at most
 * quench_max (and turns a lipid by at most quench_max radians). */
void orc_quench_project(const orc_params *p, int64_t n, const int32_t *type, const double *F, const double *T,
                        double *v, double *w);
void orc_quench_cap(const orc_ext *e, int64_t n, const int32_t *type, double dt, double *v, double *w);

/* Velocity Verlet as orc_vv_run, with the volume term in every force evaluation
 * and, when a friction rate is set, the thermostat update after each step's
 * closing half-kick; the steps are numbered step0 + 1 ... step0 + nsteps.  With
 * quench set, the velocity projection replaces the thermostat and the cap acts
 * before each drift. */
int orc_vv_run_ext(const orc_params *p, const orc_ext *e, uint64_t step0, int64_t n, double *x, double *v,
                   double *nrm, double *w, const int32_t *type, int64_t nbond, const int32_t *bonds,
                   const double *r0, double dt, int64_t nsteps, double *energies, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
