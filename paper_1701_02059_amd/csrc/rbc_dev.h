// Internal declarations shared by the HIP kernels and the host runtime of librbc.
// gfx950 only: 64-lane wavefronts, FP64 at full vector rate.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbc {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;            // threads per block for particle / cell kernels
constexpr int CHUNK = 64;             // particles per neighbour-list chunk (one wavefront)
constexpr int MAXNB = 96;             // neighbour-list rows per chunk
// per-particle type byte: the type in the low bits, and a flag for particles with bonds
// (the step kernel looks up the bond table only for those)
constexpr int TYP_MASK = 3;
constexpr int TYP_BONDED = 0x80;
constexpr int SORT_IPT = 16;          // items per thread in the radix sort
constexpr int SORT_TILE = BLOCK * SORT_IPT;
constexpr int MAX_SLOTS = 256;
constexpr int CNBR_ROW_MAX = 2048;      // cell pairs per cell before the build reports overflow
constexpr int SMAX = 2048;             // stage entries (slots) per 256-particle block
constexpr int SSTRIDE = SMAX + 32;     // stride of the blocks' stage lists (not a multiple of a large power of two)
constexpr int CANDMAX = 1024;          // candidate cells (cell-pair entries) per block while staging
constexpr int CANDBITS = 32 * CANDMAX;    // candidate-cell id range the list build sorts with a bitmap
constexpr int USTAGE = 2048;           // candidate particles staged in LDS while building a block's lists
static_assert(USTAGE <= SMAX && USTAGE < 0xffff, "a staged candidate union is the block's stage, indexed in 16 bits");
constexpr float LIST_EXTENT = 4096.0f; // largest FP32 offset (sigma) allowed in that staging
constexpr int CULLMAX = 256;           // candidate cells whose bounding spheres are staged for culling
constexpr int SCAN_TILE = 2048;        // elements per block in the segmented scans
constexpr int BRED = 12;               // doubles of per-block partial results (3 per chunk in a drift)

// error bits in SysScal::err
constexpr int ERR_NLIST = 1;          // a particle had more than MAXNB list neighbours
constexpr int ERR_CNBR = 2;           // cell-pair list capacity exceeded
constexpr int ERR_NONFINITE = 4;      // NaN / Inf in positions or velocities
constexpr int ERR_ASSIGN = 8;         // nearest-seed search found no seed

struct alignas(16) D4 {
    double x, y, z, w;
};

// A 3-vector of doubles as stored in the particle arrays that need no fourth
// component (velocity, orientation, angular velocity, force, torque): 24 B, no
// padding.  Kernels compute on D4 (ld3 / st3).
struct V3 {
    double x, y, z;
};
static_assert(sizeof(V3) == 24, "packed 3-vector");

struct alignas(16) F4 {
    float x, y, z, w;
};

struct F3 {
    float x, y, z;
};

// Per-system scalars living in device memory.
struct alignas(256) SysScal {
    unsigned long long maxdisp2;      // bits of the largest |x - x_build|^2 since the last build
    unsigned long long maxv2;         // bits of the largest |v|^2 used in a drift since the build
    unsigned long long maxdisp2p;     // bits of the largest |x - x_prune|^2 since the last prune
    unsigned long long rmax;          // bits of the largest cell radius
    int32_t err;
    int32_t rebuild;                  // this system takes part in the running cell update
    int32_t nlrows;                   // largest neighbour-list row count of the last build
    int32_t cnbr_total;
    int32_t cnbr_maxrow;
    int32_t npairs;
    int32_t pad0, pad1;
    double slo[3], shi[3];            // seed bounding box (Morton quantisation)
    double glo[3], gh[3];             // seed-grid origin and spacing
    int32_t gdim[3];
    int32_t gtot;
    double energy[9];                 // U, W, KE, sum F (3), sum r x F + tau (3)
    // volume term, from the lipid sums of the current state
    double volV;                      // V = a_L/3 sum (x_i - xbar).n_i
    double vol0;                      // V0 (set at the first evaluation when no target is given)
    double volkap;                    // dU_V/dV a_L/3: the volume force is -volkap (n_i - nbar)
    double volU;                      // U_V
    double xbar[3], nbar[3];          // lipid centroid and mean orientation
    unsigned long long step;          // drifts done since loading: numbers the thermostat's draws
    uint32_t parts_done;              // statistics blocks finished in the running pass
    uint32_t pad3;
};

// Drift statistics published to pinned host memory, one ring of STAT_RING entries
// per system indexed by the drift number: the host reads them without a copy.
constexpr int STAT_RING = 8;
// Systems of at most this many 256-particle blocks run the step kernel with each
// 64-particle chunk's list rows spread over the four waves of a block (four blocks
// per particle block): too small to fill the GPU, their step time is one wave's walk
// over its rows, which this cuts by four.
constexpr int SPLIT_MAX_BLOCKS = 32;
struct alignas(32) StepStat {
    double d2;                        // largest |x - x_build|^2 since the last build
    double v2;                        // largest |v|^2 used in a drift since the build
    double d2p;                       // largest |x - x_prune|^2 since the last prune
    unsigned long long tag;           // drift number + 1, written last (0: never written)
};

// One system (slot): sizes and device arrays.  Particle arrays are in cell-sorted
// slot order; `gid` maps a slot to the caller's particle id, `slot` the inverse.
struct SysDev {
    int32_t n, nlip, k, nchunk, gcap, cnbr_cap, ntile_p, ntile_s;
    int32_t per[3];
    int32_t kl;                                     // lipid cells: seeds [0, kl); protein cells: [kl, k)
    int32_t nsrcp;                                  // protein seed sources after the lipid ids in `lip`
    int32_t split;                                  // the step kernel spreads each chunk's rows over four waves
    double box[3];
    V3 *pos;
    uint8_t *typ;                                   // type (0 lipid, 1 junction, 2 spectrin) | TYP_BONDED
    V3 *vel, *ori, *angv, *frc, *trq;
    F3 *xb;                                         // positions at the last list build (FP32)
    F3 *xp;                                         // positions at the last prune (FP32)
    V3 *pos2;
    uint8_t *typ2;
    V3 *vel2, *ori2, *angv2;
    int32_t *gid, *gid2, *slot, *owner;
    uint64_t *key, *key2;
    uint32_t *val, *val2;
    int32_t *hist;                                  // sort histograms: tiles x 256
    D4 *seed, *seed2;                               // centroid xyz, w = cell radius
    double *sbox;                                   // per 256-seed block: the seeds' min xyz, max xyz
    int32_t *cstart, *ccount, *cstart2, *ccount2, *cmap;
    int32_t *cnbr_start, *cnbr;                     // full cell-pair CSR (k+1, cnbr_cap)
    int32_t *gstart, *gcount, *gseed, *sgcell;      // seed grid (gcap+1, gcap, k, k)
    D4 *gpos;                                       // centroids in grid order, w = seed index (k)
    int32_t *nl, *nlk;                              // neighbour lists (nchunk x MAXNB x 64), rows
    uint16_t *nl16;                                 // the same lists as stage indices (staged blocks)
    F4 *ori32;                                      // FP32 copy of the orientations, w = type bits (staging)
    F4 *ori32b;                                     // its second buffer (fused drift target; pos2 / ori2 likewise)
    int32_t *bstart, *bpart;                        // bonds by caller id (n+1, 2 nbond)
    double *br0;
    double *epart;                                  // per-chunk energy partials (nchunk x 9)
    double *vpart;                                  // per-chunk lipid sums for the volume (8 x nchunk)
    double *vred;                                   // their first-level reduction (32 x 8)
    int32_t *pairs;                                 // scratch for exporting the pair set
    int64_t pairs_cap;
    int32_t *stage, *scount;                        // per 256-particle block: staged slots (SMAX), count (-1: none)
    uint16_t *il16;                                 // pruned lists: indices into the pruned stage (0xffff pads)
    int32_t *ilk;                                   // per chunk: rows of the pruned list
    int32_t *istage, *iscount;                      // per block: the pruned stage (SMAX), count (-1: use nl)
    double *bred;                                   // per particle block: BRED partials (stats, bounding box)
    int32_t *tsum;                                  // segmented-scan tile sums
    SysScal *sc;
    StepStat *hstat;                                // this system's ring in pinned host memory
};

// Model constants, passed by value to kernels.
struct DevParams {
    double rc2[3][3];      // fl(rc*rc): exact neighbour test
    double rl2[3][3];      // (rc + 2 skin)^2 with a small relative margin: list radius
    float rl2f[3][3];      // (rc + 2 skin + 1e-3)^2 rounded up: list radius for FP32 offsets
    float rlmaxf[3];       // largest list radius (+ 1e-3) of a particle type, rounded up
    float rin2f[3][3];     // (rc + 2 inner skin + 1e-3)^2 rounded up: pruned-list radius for FP32 offsets
    float rc2lo[3][3];     // FP32 squared distances below this are inside fl(rc^2) in the exact test
    float rc2hi[3][3];     // ... and at or above this outside it; between, the FP64 test decides
    double rc_lipid, r_min, eps, mu, st0, wca_eps, wca_sig2, k_bond;
    double inv_mass[3];
    double inv_inertia;
    double cell_search;    // largest rc + 2 skin (cell-pair test slack)
    double inv_w;          // 1 / (r_c - r_min)
    double dudr_k;         // eps * zeta * pi / (r_c - r_min)
    int32_t zeta;
    int32_t vol_on;        // harmonic volume constraint
    double vol_k, vol_target, vol_a3;   // k_V, V0 (0: measured), a_L / 3
    // thermostat: v <- c v + a (r - (2^32 - 1)/2) per component, r a Philox word
    int32_t thermo_on;
    uint32_t seed_lo, seed_hi;
    int32_t pad;
    double ou_c, ou_a[3];  // translation: c = exp(-gamma dt), a per type
    double ou_cr, ou_ar;   // lipid rotation
    // velocity quenching: projection on the force after the closing kick, move cap
    int32_t quench_on;
    int32_t pad2;
    double quench_max;
};

// Block -> system maps: off[s] = first block of system s, off[nsys] = total blocks.
struct Maps {
    const int32_t *p;      // particle blocks (BLOCK particles, also 4 chunks)
    const int32_t *c;      // cell blocks
    const int32_t *g;      // seed-grid cell blocks
    const int32_t *tp;     // particle sort tiles
    const int32_t *ts;     // seed sort tiles
    const int32_t *sc;     // scan tiles over cells
    const int32_t *sg;     // scan tiles over seed-grid cells
    const int32_t *f;      // step-kernel blocks (four per particle block of a split system)
    int32_t nsys;
};

__device__ __forceinline__ int find_sys(const int32_t *off, int nsys, int b) {
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroups are dispatched to the eight XCDs in turn, and each XCD has its own L2.
// Neighbouring particle blocks stage mostly the same partners, so runs of XCD_RUN
// consecutive blocks are sent to one XCD: workgroup i, the (i / 8)-th on XCD i % 8,
// takes block ((k / XCD_RUN) * 8 + x) * XCD_RUN + k % XCD_RUN with x = i % 8 and
// k = i / 8.  A permutation of the grid's full groups of 8 XCD_RUN blocks (the
// remaining tail keeps its order), so every block is still processed once.
constexpr int XCD_RUN = 16;
__device__ __forceinline__ int xcd_group_block(int i, int n) {
    const int full = n - n % (8 * XCD_RUN);
    if (i >= full) return i;
    const int x = i & 7, k = i >> 3;
    return ((k / XCD_RUN) * 8 + x) * XCD_RUN + k % XCD_RUN;
}

// Min-image difference and squared distance exactly as the neighbour-set
// definition states: per periodic axis q = d/L, k = rint(q) (half to even),
// d - (k*L) with the product rounded; then (dx*dx + dy*dy) + dz*dz with every
// operation rounded (no contraction into fused multiply-adds).
__device__ __forceinline__ double minimg1(double d, int per, double L) {
#pragma clang fp contract(off)
    if (per) {
        double q = d / L;
        double k = __builtin_rint(q);
        double kl = k * L;
        d = d - kl;
    }
    return d;
}

__device__ __forceinline__ double dist2_exact(const SysDev &S, double xi, double yi, double zi,
                                              double xj, double yj, double zj,
                                              double &dx, double &dy, double &dz) {
#pragma clang fp contract(off)
    dx = minimg1(xi - xj, S.per[0], S.box[0]);
    dy = minimg1(yi - yj, S.per[1], S.box[1]);
    dz = minimg1(zi - zj, S.per[2], S.box[2]);
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double s = xx + yy;
    return s + zz;
}

// The same squared distance for a system without periodic axes (identical
// operations: the min-image is the identity on open axes).
__device__ __forceinline__ double dist2_open(double xi, double yi, double zi, double xj, double yj, double zj,
                                             double &dx, double &dy, double &dz) {
#pragma clang fp contract(off)
    dx = xi - xj;
    dy = yi - yj;
    dz = zi - zj;
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double s = xx + yy;
    return s + zz;
}

__device__ __forceinline__ double wrap_coord(double v, int per, double L) {
    if (!per) return v;
    double w = v - L * floor(v / L);
    if (w >= L) w -= L;
    if (w < 0) w = 0;
    return w;
}

// Loads through the global address space (the descriptor table holds generic
// pointers, which would otherwise compile to flat loads that also wait on LDS).
template <class T>
__device__ __forceinline__ T ldg(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ void stg(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}
__device__ __forceinline__ D4 ldg(const D4 *p) {
    typedef double v4d __attribute__((ext_vector_type(4)));
    const v4d v = *(const __attribute__((address_space(1))) v4d *)p;
    return D4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ V3 ldg(const V3 *p) {
    typedef const __attribute__((address_space(1))) double *gp;
    const gp q = (gp)p;
    return V3{q[0], q[1], q[2]};
}
__device__ __forceinline__ F3 ldg(const F3 *p) {
    typedef const __attribute__((address_space(1))) float *gp;
    const gp q = (gp)p;
    return F3{q[0], q[1], q[2]};
}
__device__ __forceinline__ D4 ld3(const V3 *p) {
    const V3 v = ldg(p);
    return D4{v.x, v.y, v.z, 0.0};
}
// a particle's position with its type in w
__device__ __forceinline__ D4 ldpos(const SysDev &S, int i) {
    const V3 p = ldg(S.pos + i);
    return D4{p.x, p.y, p.z, (double)(ldg(S.typ + i) & TYP_MASK)};
}
__device__ __forceinline__ void st3(V3 *p, const D4 &v) {
    typedef __attribute__((address_space(1))) double *gp;
    const gp q = (gp)p;
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
}
__device__ __forceinline__ F4 ldg(const F4 *p) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f v = *(const __attribute__((address_space(1))) v4f *)p;
    return F4{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ unsigned long long dbits(double v) {
    return (unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ double bitsd(unsigned long long b) {
    return __longlong_as_double((long long)b);
}

}  // namespace rbc

// ---------------------------------------------------------------- launch API (host)
namespace rbc {

struct LaunchCtx {
    const SysDev *S;         // device array of systems
    SysDev *Sw;              // the same array, for the kernel that swaps the drift buffers
    Maps maps;
    int32_t nblk_p, nblk_c, nblk_g, nblk_tp, nblk_ts, nblk_sc, nblk_sg, nblk_f;   // totals over systems
    int32_t nsys;
    int32_t kmin, kmax;      // fewest and most cells of a system in the launch
    DevParams prm;
    hipStream_t st;
};

// step kernels
void launch_kick_drift(const LaunchCtx &L, double dt);   // includes the per-system statistics reduction
void launch_drift_stats_swap(const LaunchCtx &L);         // statistics of a fused drift, then buffer swap
void launch_force(const LaunchCtx &L, int mixed, int energy, int kick, double dt);
void launch_reduce_energy(const LaunchCtx &L);
void launch_volume_partials(const LaunchCtx &L);          // lipid sums of the current state, per chunk
void launch_volume_reduce(const LaunchCtx &L);            // lipid sums -> V, volume force constants
void launch_scatter_state(const LaunchCtx &L, int sys, double *x, double *n, double *v, double *w, int count);
void launch_scatter_forces(const LaunchCtx &L, int sys, double *F, double *T, int count);
void launch_export_pairs(const LaunchCtx &L, int sys, int count, int32_t *out, int64_t cap, int32_t *counter);
// the allocation-free export's staging: a counter word, then pairs from byte 256
constexpr int64_t PAIR_SCRATCH_PAIRS = ((32ll << 20) - 256) / 8;
hipError_t pair_scratch_address(int device, void **out);   // this device's copy (it must be current)
void launch_zero_counter(const LaunchCtx &L, int32_t *p);
// cell update kernels (each predicated on SysScal::rebuild)
void launch_set_rebuild(const LaunchCtx &L, const unsigned long long m[4]);
void launch_restrict_maps(const LaunchCtx &L, int32_t *out);   // 7 x (nsys+1) prefix maps of the rebuilding systems
void launch_init_seeds(const LaunchCtx &L, const int32_t *const *lipids);
void launch_grid_build(const LaunchCtx &L);
void launch_assign(const LaunchCtx &L, int warm);
void launch_sort_particles(const LaunchCtx &L, int key_bits);
void launch_gather_particles(const LaunchCtx &L, int swap);   // swap: make the gathered buffers current
void launch_cell_ranges(const LaunchCtx &L);
void launch_mstep(const LaunchCtx &L);
void launch_morton_sort_seeds(const LaunchCtx &L);
void launch_block_permute(const LaunchCtx &L);
void launch_cell_bounds(const LaunchCtx &L);
void launch_cell_pairs(const LaunchCtx &L);
void launch_nlist(const LaunchCtx &L);
void launch_prune(const LaunchCtx &L);                    // pruned lists of the systems in L's particle map
void launch_mask_maps(const LaunchCtx &L, const unsigned long long m[4], int32_t *out);   // particle map of a mask
void launch_finish_update(const LaunchCtx &L, bool cells_moved);
void launch_pack(const LaunchCtx &L, int sys, const double *x, const double *n, const int32_t *type,
                 const double *v, const double *w, int count);

}  // namespace rbc
