// Voronoi ("lattice-free") cell list on gfx950: the online k-means update of the
// Spatial Searching Algorithm section, batched over every system of a context.
//
//   E-step   exact nearest centroid per particle (FP64 distance of the
//            neighbour-set definition, ties to the lower index), warm-started
//            from the particle's current cell -- the paper's warm-start
//            heuristic -- and certified by an expanding search over a uniform
//            grid of centroids (the GPU stand-in for its k-d tree).
//   sort     stable LSD radix sort of particles by owning cell (segmented per
//            system), then a gather of the particle state.
//   M-step   each centroid moves to the mean of its lipid members.
//   Morton   centroids ordered along a Morton curve (21 bits per axis), cells
//            renumbered, and particle blocks moved with their cells: the
//            two-level reordering.
//   lists    cell radii, the cell-pair list (sphere test with skin) and
//            per-particle neighbour lists in 64-particle ELL chunks.
//
// Every kernel is predicated on SysScal::rebuild so that one launch serves all
// systems that update at this step; the others are untouched.
#include "rbc_dev.h"

#include <climits>

namespace rbc {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// A running maximum that many waves raise: the atomic is issued only when the value
// read (never above the true running maximum) is smaller, so that most waves skip the
// serialised same-address atomic.
template <class T>
__device__ __forceinline__ void max_if_larger(T *p, T v) {
    if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}

__device__ __forceinline__ int wave_max_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

// Exclusive scan across the block (blockDim.x a multiple of 64, <= 1024).
__device__ int block_excl_scan(int v, int *s_w, int &total) {
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (w == 0) {
        int s = (lane < nw) ? s_w[lane] : 0;
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(s, o);
            if (lane >= o) s += y;
        }
        if (lane < nw) s_w[lane] = s;
    }
    __syncthreads();
    int base = (w > 0) ? s_w[w - 1] : 0;
    total = s_w[nw - 1];
    __syncthreads();
    return base + x - v;
}

// In-place exclusive scan of a[0..n) by one block; a[n] receives the total.
__device__ void block_scan_array(int *a, int n, int *s_w) {
    int carry = 0;
    const int per = 4;
    for (int base = 0; base < n; base += blockDim.x * per) {
        int v[per];
        int loc = 0;
        for (int q = 0; q < per; ++q) {
            int idx = base + threadIdx.x * per + q;
            v[q] = (idx < n) ? a[idx] : 0;
            loc += v[q];
        }
        int tot;
        int ex = block_excl_scan(loc, s_w, tot);
        int run = carry + ex;
        for (int q = 0; q < per; ++q) {
            int idx = base + threadIdx.x * per + q;
            if (idx < n) a[idx] = run;
            run += v[q];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) a[n] = carry;
    __syncthreads();
}

#define SYS_FROM(map) \
    const int s = find_sys(L_maps.map, L_maps.nsys, blockIdx.x); \
    const SysDev &S = Sd[s]; \
    const int lb = blockIdx.x - L_maps.map[s];

// ------------------------------------------------------------------ rebuild flags

__global__ void k_set_rebuild(const SysDev *Sd, int nsys, unsigned long long m0, unsigned long long m1,
                              unsigned long long m2, unsigned long long m3) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    unsigned long long w = (s < 64) ? m0 : (s < 128) ? m1 : (s < 192) ? m2 : m3;
    int bit = (int)((w >> (s & 63)) & 1ull);
    SysScal *sc = Sd[s].sc;
    sc->rebuild = bit;
    if (bit) {
        sc->rmax = 0ull;
        sc->nlrows = 0;
        sc->cnbr_maxrow = 0;
        sc->err &= ~(ERR_NLIST | ERR_CNBR | ERR_ASSIGN);
    }
}

// ------------------------------------------------------------------ packing

__device__ void pack_one(const SysDev &S, const double *x, const double *n, const int32_t *type, const double *v,
                       const double *w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    const int t = type[i];
    D4 p = {x[3 * i], x[3 * i + 1], x[3 * i + 2], (double)t};
    S.pos[i] = V3{p.x, p.y, p.z};
    S.typ[i] = (uint8_t)(t | (S.bstart[i + 1] > S.bstart[i] ? TYP_BONDED : 0));   // bonds by caller id = i
    S.xb[i] = F3{(float)p.x, (float)p.y, (float)p.z};
    S.xp[i] = S.xb[i];
    S.vel[i] = V3{v[3 * i], v[3 * i + 1], v[3 * i + 2]};
    if (t == 0) {
        S.ori[i] = V3{n[3 * i], n[3 * i + 1], n[3 * i + 2]};
        S.angv[i] = V3{w[3 * i], w[3 * i + 1], w[3 * i + 2]};
    } else {
        S.ori[i] = V3{0.0, 0.0, 0.0};
        S.angv[i] = V3{0.0, 0.0, 0.0};
    }
    S.frc[i] = V3{0.0, 0.0, 0.0};
    S.trq[i] = V3{0.0, 0.0, 0.0};
    S.gid[i] = i;
    S.slot[i] = i;
    S.owner[i] = -1;
}

__global__ void k_pack_multi(const SysDev *Sd, int s, const double *x, const double *n, const int32_t *type,
                             const double *v, const double *w) {
    pack_one(Sd[s], x, n, type, v, w);
}

// ------------------------------------------------------------------ seeds from lipids

// Seed j < kl starts at the position of lipid number floor(j * N_L / kl) (lipids in
// id order; `lip` lists their ids).  With a separate protein set, seed kl + j
// starts at protein number floor(j * N_P / (k - kl)), whose ids follow the lipids'
// in `lip`.  No warm start for the first assignment.
__global__ void k_init_seeds(const SysDev *Sd, Maps L_maps, const int32_t *const *lipids) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    if (c < S.k) {
        long long j;
        if (c < S.kl) j = (long long)c * S.nlip / S.kl;
        else j = S.nlip + (long long)(c - S.kl) * S.nsrcp / (S.k - S.kl);
        int g = lipids[s][j];
        D4 p = ld3(S.pos + S.slot[g]);
        p.x = wrap_coord(p.x, S.per[0], S.box[0]);
        p.y = wrap_coord(p.y, S.per[1], S.box[1]);
        p.z = wrap_coord(p.z, S.per[2], S.box[2]);
        p.w = 0.0;
        S.seed[c] = p;
    }
}

// no warm start for the first assignment after seeding
__global__ void k_clear_owner(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    int i = lb * BLOCK + threadIdx.x;
    if (i < S.n) S.owner[i] = -1;
}

// ------------------------------------------------------------------ seed grid

// Per-block bounding boxes of the (wrapped) particle positions: BRED partials 2..7.
__global__ __launch_bounds__(BLOCK) void k_bbox_partial(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    __shared__ double s_v[6][BLOCK / WAVE];
    const int i = lb * BLOCK + threadIdx.x;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (i < S.n) {
        D4 p = ld3(S.pos + i);
        double v[3] = {wrap_coord(p.x, S.per[0], S.box[0]), wrap_coord(p.y, S.per[1], S.box[1]),
                       wrap_coord(p.z, S.per[2], S.box[2])};
        for (int a = 0; a < 3; ++a) { mn[a] = v[a]; mx[a] = v[a]; }
    }
    for (int a = 0; a < 3; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = fmin(mn[a], __shfl_xor(mn[a], o));
            mx[a] = fmax(mx[a], __shfl_xor(mx[a], o));
        }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) { s_v[a][w] = mn[a]; s_v[3 + a][w] = mx[a]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        double r = s_v[a][0];
        for (int q = 1; q < BLOCK / WAVE; ++q) r = (a < 3) ? fmin(r, s_v[a][q]) : fmax(r, s_v[a][q]);
        S.bred[(size_t)lb * BRED + 2 + a] = r;
    }
}

// Per-block bounding boxes of the seeds (unwrapped centroids), 256 seeds per block.
__global__ __launch_bounds__(BLOCK) void k_seed_bbox_partial(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    __shared__ double s_v[6][BLOCK / WAVE];
    const int c = lb * BLOCK + threadIdx.x;
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (c < S.k) {
        const D4 p = S.seed[c];
        const double v[3] = {p.x, p.y, p.z};
        for (int a = 0; a < 3; ++a) { mn[a] = v[a]; mx[a] = v[a]; }
    }
    for (int a = 0; a < 3; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = fmin(mn[a], __shfl_xor(mn[a], o));
            mx[a] = fmax(mx[a], __shfl_xor(mx[a], o));
        }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) { s_v[a][w] = mn[a]; s_v[3 + a][w] = mx[a]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        double r = s_v[a][0];
        for (int q = 1; q < BLOCK / WAVE; ++q) r = (a < 3) ? fmin(r, s_v[a][q]) : fmax(r, s_v[a][q]);
        S.sbox[(size_t)lb * 6 + a] = r;
    }
}

// Bounding boxes and grid geometry, one block per system (from the per-block partials).
// Uniform grid over the seeds: cubic cells holding about one eighth of a seed each,
// but no smaller than hmin (twice the cell-pair search radius).  A cell-pair query
// walks every grid cell within its reach; on small systems a finer grid would make
// each query a long chain of dependent loads over mostly empty cells.
__global__ void k_grid_setup(const SysDev *Sd, int nsys, double hmin) {
    const SysDev &S = Sd[blockIdx.x];
    if (!S.sc->rebuild) return;
    __shared__ double s_mn[6][16], s_mx[6][16];
    double mn[6], mx[6];
    for (int a = 0; a < 6; ++a) { mn[a] = INFINITY; mx[a] = -INFINITY; }
    const int nblk = (S.n + BLOCK - 1) / BLOCK;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        const double *r = S.bred + (size_t)b * BRED + 2;
        for (int a = 0; a < 3; ++a) { mn[a] = fmin(mn[a], r[a]); mx[a] = fmax(mx[a], r[3 + a]); }
    }
    const int nsb = (S.k + BLOCK - 1) / BLOCK;
    for (int b = threadIdx.x; b < nsb; b += blockDim.x) {
        const double *r = S.sbox + (size_t)b * 6;
        for (int a = 0; a < 3; ++a) { mn[3 + a] = fmin(mn[3 + a], r[a]); mx[3 + a] = fmax(mx[3 + a], r[3 + a]); }
    }
    for (int a = 0; a < 6; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = fmin(mn[a], __shfl_xor(mn[a], o));
            mx[a] = fmax(mx[a], __shfl_xor(mx[a], o));
        }
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0)
        for (int a = 0; a < 6; ++a) { s_mn[a][w] = mn[a]; s_mx[a][w] = mx[a]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int a = 0; a < 6; ++a)
            for (int q = 1; q < nw; ++q) { mn[a] = fmin(mn[a], s_mn[a][q]); mx[a] = fmax(mx[a], s_mx[a][q]); }
        SysScal *sc = S.sc;
        double ext[3];
        for (int a = 0; a < 3; ++a) {
            // seed box for Morton keys: the box on periodic axes, the seeds' extent otherwise
            sc->slo[a] = S.per[a] ? 0.0 : mn[3 + a];
            sc->shi[a] = S.per[a] ? S.box[a] : mx[3 + a];
            if (S.per[a]) {
                sc->glo[a] = 0.0;
                ext[a] = S.box[a];
            } else {
                double lo = fmin(mn[a], mn[3 + a]), hi = fmax(mx[a], mx[3 + a]);
                if (!(lo <= hi)) { lo = 0.0; hi = 0.0; }
                double pad = 1e-6 * (hi - lo) + 1e-6;
                sc->glo[a] = lo - pad;
                ext[a] = (hi - lo) + 2.0 * pad;
            }
        }
        double cap = (double)max(1, S.gcap);
        double vol = fmax(ext[0], 1.0) * fmax(ext[1], 1.0) * fmax(ext[2], 1.0);
        double h = fmax(hmin, cbrt(vol / cap));
        int dims[3];
        for (int it = 0; it < 200; ++it) {
            double prod = 1.0;
            for (int a = 0; a < 3; ++a) {
                if (S.per[a]) dims[a] = max(1, (int)floor(ext[a] / h));
                else dims[a] = max(1, (int)ceil(ext[a] / h));
                prod *= dims[a];
            }
            if (prod <= cap) break;
            h *= 1.1;
        }
        if ((double)dims[0] * dims[1] * dims[2] > cap || !isfinite(h)) {
            dims[0] = dims[1] = dims[2] = 1;
            h = fmax(ext[0], fmax(ext[1], ext[2]));
            if (!isfinite(h) || !(h > 0.0)) h = 1.0;
        }
        for (int a = 0; a < 3; ++a) {
            sc->gdim[a] = dims[a];
            sc->gh[a] = S.per[a] ? ext[a] / dims[a] : h;
        }
        sc->gtot = dims[0] * dims[1] * dims[2];
    }
}

__device__ __forceinline__ int grid_coord(const SysScal *sc, const SysDev &S, int a, double v, double &u) {
    u = wrap_coord(v, S.per[a], S.box[a]) - sc->glo[a];
    int c = (int)floor(u / sc->gh[a]);
    c = max(0, min(c, sc->gdim[a] - 1));
    return c;
}

__global__ void k_grid_clear(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(g);
    if (!S.sc->rebuild) return;
    int g = lb * BLOCK + threadIdx.x;
    if (g < S.gcap) S.gcount[g] = 0;
}

__global__ void k_grid_count(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    if (c >= S.k) return;
    const SysScal *sc = S.sc;
    D4 p = S.seed[c];
    double u;
    int gx = grid_coord(sc, S, 0, p.x, u), gy = grid_coord(sc, S, 1, p.y, u), gz = grid_coord(sc, S, 2, p.z, u);
    int g = (gx * sc->gdim[1] + gy) * sc->gdim[2] + gz;
    S.sgcell[c] = g;
    atomicAdd(&S.gcount[g], 1);
}

// Segmented exclusive scans, three launches (tile sums, per-system scan of the
// tile sums, tile scans), specialised at compile time per array.  WHICH: 0 = seed
// grid (gcount -> gstart over gtot cells), 1 = ccount2 -> cstart2, 2 = ccount ->
// cstart, 3 = cnbr_start in place (k cells).  dst[len] receives the total.
template <int WHICH>
__device__ __forceinline__ const int *scan_src(const SysDev &S) {
    if constexpr (WHICH == 0) return S.gcount;
    else if constexpr (WHICH == 1) return S.ccount2;
    else if constexpr (WHICH == 2) return S.ccount;
    else return S.cnbr_start;
}
template <int WHICH>
__device__ __forceinline__ int *scan_dst(const SysDev &S) {
    if constexpr (WHICH == 0) return S.gstart;
    else if constexpr (WHICH == 1) return S.cstart2;
    else if constexpr (WHICH == 2) return S.cstart;
    else return S.cnbr_start;
}
template <int WHICH>
__device__ __forceinline__ int scan_len(const SysDev &S) {
    if constexpr (WHICH == 0) return S.sc->gtot;
    else return S.k;
}

template <int WHICH>
__global__ __launch_bounds__(BLOCK) void k_scan_a(const SysDev *Sd, Maps L_maps) {
    const int32_t *map = WHICH == 0 ? L_maps.sg : L_maps.sc;
    const int s = find_sys(map, L_maps.nsys, blockIdx.x);
    const SysDev &S = Sd[s];
    if (!S.sc->rebuild) return;
    const int tile = blockIdx.x - map[s];
    const int *src = scan_src<WHICH>(S);
    const int len = scan_len<WHICH>(S);
    __shared__ int s_w[16];
    constexpr int per = SCAN_TILE / BLOCK;
    int loc = 0;
    for (int q = 0; q < per; ++q) {
        const int idx = tile * SCAN_TILE + threadIdx.x * per + q;
        if (idx < len) loc += src[idx];
    }
    int tot;
    (void)block_excl_scan(loc, s_w, tot);
    if (threadIdx.x == 0) S.tsum[tile] = tot;
}

template <int WHICH>
__global__ __launch_bounds__(1024) void k_scan_b(const SysDev *Sd) {
    const SysDev &S = Sd[blockIdx.x];
    if (!S.sc->rebuild) return;
    __shared__ int s_w[16];
    const int ntile = (scan_len<WHICH>(S) + SCAN_TILE - 1) / SCAN_TILE;
    block_scan_array(S.tsum, ntile, s_w);
}

template <int WHICH>
__global__ __launch_bounds__(BLOCK) void k_scan_c(const SysDev *Sd, Maps L_maps) {
    const int32_t *map = WHICH == 0 ? L_maps.sg : L_maps.sc;
    const int s = find_sys(map, L_maps.nsys, blockIdx.x);
    const SysDev &S = Sd[s];
    if (!S.sc->rebuild) return;
    const int tile = blockIdx.x - map[s];
    const int *src = scan_src<WHICH>(S);
    int *dst = scan_dst<WHICH>(S);
    const int len = scan_len<WHICH>(S);
    const int ntile = (len + SCAN_TILE - 1) / SCAN_TILE;
    if (tile >= ntile) return;
    __shared__ int s_w[16];
    constexpr int per = SCAN_TILE / BLOCK;
    int v[per];
    int loc = 0;
    for (int q = 0; q < per; ++q) {
        const int idx = tile * SCAN_TILE + threadIdx.x * per + q;
        v[q] = (idx < len) ? src[idx] : 0;
        loc += v[q];
    }
    int tot;
    int run = S.tsum[tile] + block_excl_scan(loc, s_w, tot);
    for (int q = 0; q < per; ++q) {
        const int idx = tile * SCAN_TILE + threadIdx.x * per + q;
        if (idx < len) dst[idx] = run;
        run += v[q];
    }
    if (tile == ntile - 1 && threadIdx.x == 0) dst[len] = S.tsum[ntile];
}

template <int WHICH>
static void launch_scan_t(const LaunchCtx &L) {
    const int nblk = WHICH == 0 ? L.nblk_sg : L.nblk_sc;
    hipLaunchKernelGGL(k_scan_a<WHICH>, dim3(nblk), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_scan_b<WHICH>, dim3(L.nsys), dim3(1024), 0, L.st, L.S);
    hipLaunchKernelGGL(k_scan_c<WHICH>, dim3(nblk), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

static void launch_scan(const LaunchCtx &L, int which) {
    switch (which) {
        case 0: launch_scan_t<0>(L); break;
        case 1: launch_scan_t<1>(L); break;
        case 2: launch_scan_t<2>(L); break;
        default: launch_scan_t<3>(L); break;
    }
}

__global__ void k_grid_fill(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    if (c >= S.k) return;
    int g = S.sgcell[c];
    int p = S.gstart[g] + atomicAdd(&S.gcount[g], 1);
    S.gseed[p] = c;
}

// Seeds inside a grid cell in ascending index order (deterministic scans).
__global__ void k_grid_sortcells(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(g);
    if (!S.sc->rebuild) return;
    int g = lb * BLOCK + threadIdx.x;
    if (g >= S.sc->gtot) return;
    int b = S.gstart[g], e = S.gstart[g + 1];
    for (int i = b + 1; i < e; ++i) {
        int v = S.gseed[i];
        int j = i - 1;
        while (j >= b && S.gseed[j] > v) { S.gseed[j + 1] = S.gseed[j]; --j; }
        S.gseed[j + 1] = v;
    }
    // centroid positions in grid order, seed index in w (one load per candidate in the E-step)
    for (int q = b; q < e; ++q) {
        const int sd = S.gseed[q];
        const D4 c = S.seed[sd];
        S.gpos[q] = D4{c.x, c.y, c.z, (double)sd};
    }
}

void launch_grid_build(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_bbox_partial, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_seed_bbox_partial, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_grid_setup, dim3(L.nsys), dim3(1024), 0, L.st, L.S, L.nsys, 2.0 * L.prm.cell_search);
    hipLaunchKernelGGL(k_grid_clear, dim3(L.nblk_g), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_grid_count, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
    launch_scan(L, 0);
    hipLaunchKernelGGL(k_grid_clear, dim3(L.nblk_g), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_grid_fill, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_grid_sortcells, dim3(L.nblk_g), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

// ------------------------------------------------------------------ E-step

// Per-axis window of grid offsets searched at radius r: open axes are clipped at
// the grid edge, periodic axes stop growing once every cell is covered.
__device__ __forceinline__ void axis_window(int c, int dim, int per, int r, int &lo, int &hi) {
    if (per) {
        int half = (dim - 1) / 2;
        lo = -min(r, half);
        hi = min(r, dim - 1 - half);
    } else {
        lo = max(-r, -c);
        hi = min(r, dim - 1 - c);
    }
}

// Nearest centroid among seeds [slo, shi) (ties: lower index).
__device__ int nearest_seed(const SysDev &S, const SysScal *sc, double xi, double yi, double zi, int warm,
                            int slo, int shi, double &bestd2) {
    int best = -1;
    bestd2 = INFINITY;
    double dx, dy, dz;
    const unsigned span = (unsigned)(shi - slo);
    if (warm >= 0 && (unsigned)(warm - slo) < span) {
        D4 c = S.seed[warm];
        bestd2 = dist2_exact(S, xi, yi, zi, c.x, c.y, c.z, dx, dy, dz);
        best = warm;
    }
    double u[3];
    int cc[3];
    cc[0] = grid_coord(sc, S, 0, xi, u[0]);
    cc[1] = grid_coord(sc, S, 1, yi, u[1]);
    cc[2] = grid_coord(sc, S, 2, zi, u[2]);
    int plo[3] = {1, 1, 1}, phi[3] = {-1, -1, -1};
    int rmax = max(sc->gdim[0], max(sc->gdim[1], sc->gdim[2]));
    for (int r = 0; r <= rmax; ++r) {
        int lo[3], hi[3];
        bool grew = false;
        for (int a = 0; a < 3; ++a) {
            axis_window(cc[a], sc->gdim[a], S.per[a], r, lo[a], hi[a]);
            if (lo[a] < plo[a] || hi[a] > phi[a]) grew = true;
        }
        if (!grew) break;   // every cell visited
        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
            bool nx = (ox < plo[0] || ox > phi[0]);
            int gx = cc[0] + ox;
            if (S.per[0]) gx = (gx % sc->gdim[0] + sc->gdim[0]) % sc->gdim[0];
            for (int oy = lo[1]; oy <= hi[1]; ++oy) {
                bool ny = nx || (oy < plo[1] || oy > phi[1]);
                int gy = cc[1] + oy;
                if (S.per[1]) gy = (gy % sc->gdim[1] + sc->gdim[1]) % sc->gdim[1];
                // the column's cells not visited at a smaller radius: the whole z window
                // where the column is new, else the rows below and above the previous
                // window; each a run of consecutive grid cells (split where a periodic z
                // axis wraps), whose seeds are one range of gpos
                int ra[2], rb[2], nr = 0;
                if (ny) {
                    ra[0] = lo[2]; rb[0] = hi[2]; nr = 1;
                } else {
                    if (lo[2] < plo[2]) { ra[nr] = lo[2]; rb[nr] = min(hi[2], plo[2] - 1); ++nr; }
                    if (hi[2] > phi[2]) { ra[nr] = max(lo[2], phi[2] + 1); rb[nr] = hi[2]; ++nr; }
                }
                const int nzg = sc->gdim[2], base = (gx * sc->gdim[1] + gy) * nzg;
                for (int k = 0; k < nr; ++k) {
                    int za = cc[2] + ra[k], zb = cc[2] + rb[k];
                    int z2a = 0, z2b = -1;                // the wrapped part, if any
                    if (S.per[2]) {                       // the window spans at most nzg rows
                        if (za < 0) {
                            if (zb < 0) { za += nzg; zb += nzg; }
                            else { z2a = 0; z2b = zb; za += nzg; zb = nzg - 1; }
                        } else if (zb >= nzg) {
                            if (za >= nzg) { za -= nzg; zb -= nzg; }
                            else { z2a = 0; z2b = zb - nzg; zb = nzg - 1; }
                        }
                    }
                    for (int part = 0; part < 2; ++part) {
                        const int a0 = part ? z2a : za, a1 = part ? z2b : zb;
                        if (a1 < a0) continue;
                        const int qe = ldg(S.gstart + base + a1 + 1);
                        for (int q = ldg(S.gstart + base + a0); q < qe; ++q) {
                            const D4 c = ldg(S.gpos + q);
                            const int sd = (int)c.w;
                            if ((unsigned)(sd - slo) >= span) continue;   // the other particle set's cells
                            double d2 = dist2_exact(S, xi, yi, zi, c.x, c.y, c.z, dx, dy, dz);
                            if (d2 < bestd2 || (d2 == bestd2 && sd < best)) { bestd2 = d2; best = sd; }
                        }
                    }
                }
            }
        }
        for (int a = 0; a < 3; ++a) { plo[a] = lo[a]; phi[a] = hi[a]; }
        // distance from the particle to the nearest cell not yet visited
        double m = INFINITY;
        for (int a = 0; a < 3; ++a) {
            int dim = sc->gdim[a];
            bool full = S.per[a] ? (hi[a] - lo[a] + 1 >= dim) : false;
            if (full) continue;
            bool lo_open = S.per[a] ? true : (cc[a] + lo[a] > 0);
            bool hi_open = S.per[a] ? true : (cc[a] + hi[a] < dim - 1);
            if (lo_open) m = fmin(m, u[a] - (double)(cc[a] + lo[a]) * sc->gh[a]);
            if (hi_open) m = fmin(m, (double)(cc[a] + hi[a] + 1) * sc->gh[a] - u[a]);
        }
        if (m == INFINITY) break;
        if (best >= 0 && m > 0.0) {
            double mm = m * (1.0 - 1e-9);
            if (bestd2 < mm * mm) break;
        }
    }
    return best;
}

__global__ void k_assign(const SysDev *Sd, Maps L_maps, int warm) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    int i = lb * BLOCK + threadIdx.x;
    if (i >= S.n) return;
    D4 p = ldpos(S, i);
    double d2;
    // lipids search cells [0, kl), protein beads [kl, k) (all cells when kl == k)
    const bool lipid_set = (p.w == 0.0) || S.kl == S.k;
    const int slo = lipid_set ? 0 : S.kl, shi = lipid_set ? S.kl : S.k;
    int best = nearest_seed(S, S.sc, p.x, p.y, p.z, warm ? S.owner[i] : -1, slo, shi, d2);
    if (best < 0) { atomicOr(&S.sc->err, ERR_ASSIGN); best = 0; }
    S.key[i] = (uint64_t)best;
    S.val[i] = (uint32_t)i;
}

void launch_assign(const LaunchCtx &L, int warm) {
    hipLaunchKernelGGL(k_assign, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, warm);
}

// ------------------------------------------------------------------ segmented stable radix sort

// kind 0: particles (S.n keys, tiles map tp); kind 1: seeds (S.k keys, map ts).
__global__ __launch_bounds__(BLOCK) void k_sort_hist(const SysDev *Sd, Maps L_maps, int kind, int pass) {
    const int32_t *map = kind ? L_maps.ts : L_maps.tp;
    const int s = find_sys(map, L_maps.nsys, blockIdx.x);
    const SysDev &S = Sd[s];
    if (!S.sc->rebuild) return;
    const int tile = blockIdx.x - map[s];
    const int cnt = kind ? S.k : S.n;
    const uint64_t *keys = (pass & 1) ? S.key2 : S.key;
    const int shift = 8 * pass;
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = tile * SORT_TILE;
    for (int r = 0; r < SORT_IPT; ++r) {
        int idx = base + r * BLOCK + threadIdx.x;
        if (idx < cnt) atomicAdd(&h[(int)((keys[idx] >> shift) & 255ull)], 1);
    }
    __syncthreads();
    S.hist[tile * 256 + threadIdx.x] = h[threadIdx.x];
}

// Column scan of the tile histograms: one block per (system, digit) turns the
// digit's per-tile counts into exclusive tile offsets within the digit and leaves
// the digit's total after the last tile row (the scatter adds the digit bases).
__global__ __launch_bounds__(256) void k_sort_scan(const SysDev *Sd, int kind) {
    const SysDev &S = Sd[blockIdx.x >> 8];
    if (!S.sc->rebuild) return;
    const int d = blockIdx.x & 255;
    const int cnt = kind ? S.k : S.n;
    const int ntile = (cnt + SORT_TILE - 1) / SORT_TILE;
    __shared__ int s_w[16];
    int carry = 0;
    for (int t0 = 0; t0 < ntile; t0 += 256) {
        const int t = t0 + (int)threadIdx.x;
        const int v = t < ntile ? S.hist[t * 256 + d] : 0;
        int tot;
        const int ex = block_excl_scan(v, s_w, tot);
        if (t < ntile) S.hist[t * 256 + d] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) S.hist[ntile * 256 + d] = carry;
}

__global__ __launch_bounds__(BLOCK) void k_sort_scatter(const SysDev *Sd, Maps L_maps, int kind, int pass) {
    const int32_t *map = kind ? L_maps.ts : L_maps.tp;
    const int s = find_sys(map, L_maps.nsys, blockIdx.x);
    const SysDev &S = Sd[s];
    if (!S.sc->rebuild) return;
    const int tile = blockIdx.x - map[s];
    const int cnt = kind ? S.k : S.n;
    const uint64_t *kin = (pass & 1) ? S.key2 : S.key;
    const uint32_t *vin = (pass & 1) ? S.val2 : S.val;
    uint64_t *kout = (pass & 1) ? S.key : S.key2;
    uint32_t *vout = (pass & 1) ? S.val : S.val2;
    const int shift = 8 * pass;
    __shared__ int s_base[256];
    __shared__ int s_cnt[BLOCK / WAVE][256];
    __shared__ int s_w[16];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    {
        const int ntile = (cnt + SORT_TILE - 1) / SORT_TILE;
        int tot;
        const int digit_base = block_excl_scan(S.hist[ntile * 256 + tid], s_w, tot);
        s_base[tid] = S.hist[tile * 256 + tid] + digit_base;
    }
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < SORT_IPT; ++r) {
        for (int q = tid; q < (BLOCK / WAVE) * 256; q += BLOCK) s_cnt[q >> 8][q & 255] = 0;
        __syncthreads();
        int idx = tile * SORT_TILE + r * BLOCK + tid;
        bool valid = idx < cnt;
        uint64_t k = valid ? kin[idx] : 0ull;
        uint32_t v = valid ? vin[idx] : 0u;
        int d = (int)((k >> shift) & 255ull);
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            unsigned long long mb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? mb : ~mb;
        }
        int rank = __popcll(peers & lt);
        if (valid && rank == 0) s_cnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pre = 0;
            for (int q = 0; q < w; ++q) pre += s_cnt[q][d];
            int pos = s_base[d] + pre + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        int add = 0;
        for (int q = 0; q < BLOCK / WAVE; ++q) add += s_cnt[q][tid];
        s_base[tid] += add;
        __syncthreads();
    }
}

static void sort_segments(const LaunchCtx &L, int kind, int key_bits) {
    int passes = (key_bits + 7) / 8;
    if (passes & 1) ++passes;           // even: the result lands back in key/val
    int nblk = kind ? L.nblk_ts : L.nblk_tp;
    for (int p = 0; p < passes; ++p) {
        hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(BLOCK), 0, L.st, L.S, L.maps, kind, p);
        hipLaunchKernelGGL(k_sort_scan, dim3(L.nsys * 256), dim3(256), 0, L.st, L.S, kind);
        hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(BLOCK), 0, L.st, L.S, L.maps, kind, p);
    }
}

void launch_sort_particles(const LaunchCtx &L, int key_bits) { sort_segments(L, 0, key_bits); }

// ------------------------------------------------------------------ gather / commit

// new slot j takes old slot val[j]; owner of j is key[j]
__global__ void k_gather(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    int j = lb * BLOCK + threadIdx.x;
    if (j >= S.n) return;
    int src = (int)S.val[j];
    S.pos2[j] = S.pos[src];
    S.typ2[j] = S.typ[src];
    S.vel2[j] = S.vel[src];
    S.ori2[j] = S.ori[src];
    S.angv2[j] = S.angv[src];
    S.gid2[j] = S.gid[src];
}

// copy the gathered state back; owner from key (mode 0) or val (mode 1)
__global__ void k_commit(const SysDev *Sd, Maps L_maps, int mode) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    int j = lb * BLOCK + threadIdx.x;
    if (j >= S.n) return;
    S.pos[j] = S.pos2[j];
    S.typ[j] = S.typ2[j];
    S.vel[j] = S.vel2[j];
    S.ori[j] = S.ori2[j];
    S.angv[j] = S.angv2[j];
    int g = S.gid2[j];
    S.gid[j] = g;
    S.slot[g] = j;
    S.owner[j] = mode ? (int)S.val[j] : (int)S.key[j];
}

// The gathered state becomes current by swapping the buffer pointers of the
// rebuilding systems in the descriptor table (each update swaps twice, so the
// host's copy of the table stays valid); only the id maps and owners are written.
__global__ void k_swap_state(SysDev *Sd, int nsys) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsys) return;
    SysDev &S = Sd[s];
    if (S.n <= 0 || !S.sc->rebuild) return;
    V3 *u;
    u = S.pos; S.pos = S.pos2; S.pos2 = u;
    uint8_t *y = S.typ; S.typ = S.typ2; S.typ2 = y;
    u = S.vel; S.vel = S.vel2; S.vel2 = u;
    u = S.ori; S.ori = S.ori2; S.ori2 = u;
    u = S.angv; S.angv = S.angv2; S.angv2 = u;
    int32_t *g = S.gid; S.gid = S.gid2; S.gid2 = g;
}

__global__ void k_commit_ids(const SysDev *Sd, Maps L_maps, int mode) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    int j = lb * BLOCK + threadIdx.x;
    if (j >= S.n) return;
    S.slot[S.gid[j]] = j;
    S.owner[j] = mode ? (int)S.val[j] : (int)S.key[j];
}

static void swap_and_commit(const LaunchCtx &L, int mode) {
    hipLaunchKernelGGL(k_swap_state, dim3((L.nsys + 63) / 64), dim3(64), 0, L.st, L.Sw, L.nsys);
    hipLaunchKernelGGL(k_commit_ids, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, mode);
}

void launch_gather_particles(const LaunchCtx &L, int swap) {
    hipLaunchKernelGGL(k_gather, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps);
    if (swap) swap_and_commit(L, 0);
    else hipLaunchKernelGGL(k_commit, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, 0);
}

// ------------------------------------------------------------------ cell ranges

// Cell ranges from the owners, which the sort left in ascending order: where the
// owner changes between slots j-1 and j, every cell in between starts at j.
__global__ void k_cell_starts(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    const int j = lb * BLOCK + threadIdx.x;
    if (j >= S.n) return;
    const int o = S.owner[j];
    const int prev = j > 0 ? S.owner[j - 1] : -1;
    for (int c = prev + 1; c <= o; ++c) S.cstart[c] = j;
    if (j == S.n - 1)
        for (int c = o + 1; c <= S.k; ++c) S.cstart[c] = S.n;
}

__global__ void k_cell_counts(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    const int c = lb * BLOCK + threadIdx.x;
    if (c < S.k) S.ccount[c] = S.cstart[c + 1] - S.cstart[c];
}

void launch_cell_ranges(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_cell_starts, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_cell_counts, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

// ------------------------------------------------------------------ M-step

// Each centroid with lipid members moves by the mean min-image offset of those
// members (summed in slot order); centroids without lipids stay; periodic axes wrap.
// Cells of a separate protein set (index >= kl) average their protein members.
__global__ void k_mstep(const SysDev *Sd, Maps L_maps) {
#pragma clang fp contract(off)
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    if (c >= S.k) return;
    D4 sd = S.seed[c];
    double sx = 0, sy = 0, sz = 0;
    int cnt = 0;
    const bool lipid_cell = c < S.kl;
    int b = S.cstart[c], e = b + S.ccount[c];
    for (int i = b; i < e; ++i) {
        D4 p = ldpos(S, i);
        if ((p.w == 0.0) != lipid_cell) continue;
        double dx, dy, dz;
        (void)dist2_exact(S, p.x, p.y, p.z, sd.x, sd.y, sd.z, dx, dy, dz);
        sx += dx; sy += dy; sz += dz;
        ++cnt;
    }
    if (cnt > 0) {
        double inv = (double)cnt;
        double v[3] = {sd.x + sx / inv, sd.y + sy / inv, sd.z + sz / inv};
        for (int a = 0; a < 3; ++a)
            if (S.per[a]) v[a] = v[a] - S.box[a] * floor(v[a] / S.box[a]);
        sd.x = v[0]; sd.y = v[1]; sd.z = v[2];
        S.seed[c] = sd;
    }
}

void launch_mstep(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_mstep, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

// ------------------------------------------------------------------ Morton order of centroids

__global__ void k_seed_bbox(const SysDev *Sd, int nsys) {
    const SysDev &S = Sd[blockIdx.x];
    if (!S.sc->rebuild) return;
    __shared__ double s_mn[3][16], s_mx[3][16];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    const int nsb = (S.k + BLOCK - 1) / BLOCK;
    for (int b = threadIdx.x; b < nsb; b += blockDim.x) {
        const double *r = S.sbox + (size_t)b * 6;
        for (int a = 0; a < 3; ++a) { mn[a] = fmin(mn[a], r[a]); mx[a] = fmax(mx[a], r[3 + a]); }
    }
    for (int a = 0; a < 3; ++a)
        for (int o = 32; o > 0; o >>= 1) {
            mn[a] = fmin(mn[a], __shfl_xor(mn[a], o));
            mx[a] = fmax(mx[a], __shfl_xor(mx[a], o));
        }
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    if (lane == 0) for (int a = 0; a < 3; ++a) { s_mn[a][w] = mn[a]; s_mx[a][w] = mx[a]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int a = 0; a < 3; ++a) {
            for (int q = 1; q < nw; ++q) { mn[a] = fmin(mn[a], s_mn[a][q]); mx[a] = fmax(mx[a], s_mx[a][q]); }
            S.sc->slo[a] = S.per[a] ? 0.0 : mn[a];
            S.sc->shi[a] = S.per[a] ? S.box[a] : mx[a];
        }
    }
}

// 21-bit quantisation per axis, bits interleaved x (most significant), y, z; bit 63
// marks a protein-set cell, so lipid cells keep the indices below kl.
__global__ void k_morton(const SysDev *Sd, Maps L_maps) {
#pragma clang fp contract(off)
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    if (c >= S.k) return;
    D4 p = S.seed[c];
    double v[3] = {p.x, p.y, p.z};
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
        double ext = S.sc->shi[a] - S.sc->slo[a];
        if (!(ext > 0.0)) { q[a] = 0; continue; }
        double f = (v[a] - S.sc->slo[a]) / ext;
        double t = floor(f * 2097152.0);
        if (t < 0.0) t = 0.0;
        if (t > 2097151.0) t = 2097151.0;
        q[a] = (uint64_t)t;
    }
    uint64_t key = 0;
    for (int b = 20; b >= 0; --b)
        key = (key << 3) | (((q[0] >> b) & 1ull) << 2) | (((q[1] >> b) & 1ull) << 1) | ((q[2] >> b) & 1ull);
    if (c >= S.kl) key |= 1ull << 63;
    S.key[c] = key;
    S.val[c] = (uint32_t)c;
}

// new cell c' takes old cell val[c']; cmap[old] = new
__global__ void k_seed_permute(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    if (c >= S.k) return;
    int old = (int)S.val[c];
    S.seed2[c] = S.seed[old];
    S.ccount2[c] = S.ccount[old];
    S.cmap[old] = c;
}

void launch_morton_sort_seeds(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_seed_bbox_partial, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
    hipLaunchKernelGGL(k_seed_bbox, dim3(L.nsys), dim3(1024), 0, L.st, L.S, L.nsys);
    hipLaunchKernelGGL(k_morton, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
    sort_segments(L, 1, 64);
    hipLaunchKernelGGL(k_seed_permute, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
    launch_scan(L, 1);
}

// particles move with their renumbered cells, keeping their order inside a cell
__global__ void k_block_permute(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    int j = lb * BLOCK + threadIdx.x;
    if (j >= S.n) return;
    int c = S.owner[j];
    int cn = S.cmap[c];
    int dst = S.cstart2[cn] + (j - S.cstart[c]);
    S.pos2[dst] = S.pos[j];
    S.typ2[dst] = S.typ[j];
    S.vel2[dst] = S.vel[j];
    S.ori2[dst] = S.ori[j];
    S.angv2[dst] = S.angv[j];
    S.gid2[dst] = S.gid[j];
    S.val[dst] = (uint32_t)cn;
}

__global__ void k_cell_commit(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    if (c >= S.k) return;
    S.seed[c] = S.seed2[c];
    S.ccount[c] = S.ccount2[c];
    S.cstart[c] = S.cstart2[c];
    if (c == S.k - 1) S.cstart[S.k] = S.cstart2[S.k];
}

void launch_block_permute(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_block_permute, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps);
    swap_and_commit(L, 1);
    hipLaunchKernelGGL(k_cell_commit, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

// ------------------------------------------------------------------ cell radii and cell pairs

__global__ void k_cell_bounds(const SysDev *Sd, Maps L_maps) {
    SYS_FROM(c);
    if (!S.sc->rebuild) return;
    int c = lb * BLOCK + threadIdx.x;
    double R = 0.0;
    if (c < S.k) {
        D4 sd = S.seed[c];
        double r2 = 0.0;
        int b = S.cstart[c], e = b + S.ccount[c];
        for (int i = b; i < e; ++i) {
            D4 p = ld3(S.pos + i);
            double dx, dy, dz;
            r2 = fmax(r2, dist2_exact(S, p.x, p.y, p.z, sd.x, sd.y, sd.z, dx, dy, dz));
        }
        R = sqrt(r2);
        S.seed[c].w = R;
    }
    for (int o = 32; o > 0; o >>= 1) R = fmax(R, __shfl_xor(R, o));
    if ((threadIdx.x & 63) == 0 && c - (int)(threadIdx.x & 63) < S.k) max_if_larger(&S.sc->rmax, dbits(R));
}

// The query window of cell A on the seed grid: per axis the grid rows within
// R_A + R_max + search of its centroid (a periodic axis wraps; a window that covers
// the period, or a non-finite bound, takes the whole axis).  Along z, whose grid cells
// are consecutive in the grid's linear order, the window is one or two runs of grid
// cells (two where it wraps), so that the seeds of a run are one range of `gseed`.
struct QWin {
    int lo[2], n[2];          // x and y: first row (before wrapping) and row count
    int za[2], zb[2], nz;     // z runs [za, zb] (wrapped), in walk order
};
__device__ __forceinline__ QWin query_window(const SysDev &S, const SysScal *sc, const D4 &ca, double search) {
    const double rho = ca.w + bitsd(sc->rmax) + search + 1e-9;
    const double xa[3] = {ca.x, ca.y, ca.z};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        double u = wrap_coord(xa[a], S.per[a], S.box[a]) - sc->glo[a];
        int dim = sc->gdim[a];
        double fl = floor((u - rho) / sc->gh[a]), fh = floor((u + rho) / sc->gh[a]);
        if (!(fl > -1e9 && fh < 1e9)) { fl = 0.0; fh = (double)(dim - 1); }   // non-finite: scan the axis
        int l = (int)fl;
        int h = (int)fh;
        if (S.per[a]) {
            if (h - l + 1 >= dim) { l = 0; h = dim - 1; }
        } else {
            l = max(l, 0);
            h = min(h, dim - 1);
        }
        lo[a] = l;
        hi[a] = h;
    }
    QWin w;
    for (int a = 0; a < 2; ++a) {
        w.lo[a] = lo[a];
        w.n[a] = max(0, hi[a] - lo[a] + 1);
    }
    const int dz = sc->gdim[2];
    w.nz = 0;
    if (hi[2] >= lo[2]) {
        if (lo[2] < 0) {                  // periodic: the rows below 0 are the top ones, walked first
            w.za[0] = lo[2] + dz; w.zb[0] = dz - 1;
            w.za[1] = 0; w.zb[1] = hi[2];
            w.nz = 2;
        } else if (hi[2] >= dz) {
            w.za[0] = lo[2]; w.zb[0] = dz - 1;
            w.za[1] = 0; w.zb[1] = hi[2] - dz;
            w.nz = 2;
        } else {
            w.za[0] = lo[2]; w.zb[0] = hi[2];
            w.nz = 1;
        }
    }
    return w;
}

// The linear index of grid column (x row, y row) of the window, wrapped on periodic axes.
__device__ __forceinline__ int window_column(const SysDev &S, const SysScal *sc, const QWin &w, int ix, int iy) {
    int gx = w.lo[0] + ix, gy = w.lo[1] + iy;
    if (S.per[0]) gx = ((gx % sc->gdim[0]) + sc->gdim[0]) % sc->gdim[0];
    if (S.per[1]) gy = ((gy % sc->gdim[1]) + sc->gdim[1]) % sc->gdim[1];
    return (gx * sc->gdim[1] + gy) * sc->gdim[2];
}

// Whether seed B pairs with cell A (centroid ca, radius ca.w).
__device__ __forceinline__ bool cell_pair_test(const SysDev &S, const D4 &ca, const D4 &cb, double search) {
    double dx, dy, dz;
    const double d = sqrt(dist2_exact(S, ca.x, ca.y, ca.z, cb.x, cb.y, cb.z, dx, dy, dz));
    return d <= ca.w + cb.w + search + 1e-9;
}

// Cells B paired with A (as below), one thread per cell: the serial walk of the
// window, a column's z runs at a time.  mode 0 counts, mode 1 writes (grid-scan order).
__device__ int cell_query_serial(const SysDev &S, const SysScal *sc, int A, double search, int mode, int *out, int cap) {
    const D4 ca = S.seed[A];
    const QWin w = query_window(S, sc, ca, search);
    int cnt = 0;
    for (int ix = 0; ix < w.n[0]; ++ix)
        for (int iy = 0; iy < w.n[1]; ++iy) {
            const int base = window_column(S, sc, w, ix, iy);
            for (int r = 0; r < w.nz; ++r) {
                const int qe = ldg(S.gstart + base + w.zb[r] + 1);
                for (int q = ldg(S.gstart + base + w.za[r]); q < qe; ++q) {
                    const int B = ldg(S.gseed + q);
                    if (cell_pair_test(S, ca, ldg(S.seed + B), search)) {
                        if (mode && cnt < cap) out[cnt] = B;
                        ++cnt;
                    }
                }
            }
        }
    return cnt;
}

// Cells B paired with A: |minimg(c_A - c_B)| <= R_A + R_B + search + 1e-9 with
// search = largest (rc + 2 skin).  One wavefront per cell A: the window's grid columns
// (x slowest) are taken 64 at a time, lane l scanning the seeds of the l-th one's z
// runs.  With `out`, the hits are written in that scan order (an exclusive scan of the
// lanes' counts places each lane's hits), so the row is the same as a serial walk of
// the window would give.  Returns the row's length on every lane.
__device__ int cell_query_wave(const SysDev &S, const SysScal *sc, int A, double search, int32_t *out, int cap) {
    const int lane = threadIdx.x & (WAVE - 1);
    const D4 ca = S.seed[A];
    const QWin w = query_window(S, sc, ca, search);
    const int W = w.n[0] * w.n[1];
    int total = 0;
    for (int w0 = 0; w0 < W; w0 += WAVE) {
        const int wi = w0 + lane;
        int qb[2] = {0, 0}, qe[2] = {0, 0};
        if (wi < W) {
            const int base = window_column(S, sc, w, wi / w.n[1], wi % w.n[1]);
            for (int r = 0; r < w.nz; ++r) {
                qb[r] = ldg(S.gstart + base + w.za[r]);
                qe[r] = ldg(S.gstart + base + w.zb[r] + 1);
            }
        }
        int cnt = 0;
        for (int r = 0; r < 2; ++r)
            for (int q = qb[r]; q < qe[r]; ++q)
                if (cell_pair_test(S, ca, ldg(S.seed + ldg(S.gseed + q)), search)) ++cnt;
        // inclusive scan of the lanes' counts
        int inc = cnt;
        for (int o = 1; o < WAVE; o <<= 1) {
            const int y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        if (out && cnt > 0) {
            int k = total + inc - cnt;
            for (int r = 0; r < 2; ++r)
                for (int q = qb[r]; q < qe[r]; ++q) {
                    const int B = ldg(S.gseed + q);
                    if (cell_pair_test(S, ca, ldg(S.seed + B), search)) {
                        if (k < cap) out[k] = B;
                        ++k;
                    }
                }
        }
        total += __shfl(inc, WAVE - 1);
    }
    return total;
}

// Cell-pair kernels.  Systems of at least CQ_SERIAL_MIN cells take one thread per
// cell (there are enough threads to hide the serial walk's latency); smaller ones
// give each cell a wavefront, CQ_WAVE consecutive cells per wavefront in turn and
// CQ_BLOCKS blocks per 256-cell block of the cell map.  Both write the same rows.
constexpr int CQ_WAVE = 1;
constexpr int CQ_BLOCKS = BLOCK / ((BLOCK / WAVE) * CQ_WAVE);
constexpr int CQ_SERIAL_MIN = 20000;

__global__ __launch_bounds__(BLOCK) void k_cnbr_count_serial(const SysDev *Sd, Maps L_maps, double search) {
    SYS_FROM(c);
    if (!S.sc->rebuild || S.k < CQ_SERIAL_MIN) return;
    const int c = lb * BLOCK + threadIdx.x;
    int n = 0;
    if (c < S.k) {
        n = cell_query_serial(S, S.sc, c, search, 0, nullptr, 0);
        if (n > CNBR_ROW_MAX) {          // keeps the scanned total inside int32
            atomicOr(&S.sc->err, ERR_CNBR);
            n = 0;
        }
        S.cnbr_start[c] = n;
    }
    const int m = wave_max_int(n);
    if ((threadIdx.x & 63) == 0 && m > 0) max_if_larger(&S.sc->cnbr_maxrow, m);
}

__global__ __launch_bounds__(BLOCK) void k_cnbr_fill_serial(const SysDev *Sd, Maps L_maps, double search) {
    SYS_FROM(c);
    if (!S.sc->rebuild || S.k < CQ_SERIAL_MIN) return;
    const int c = lb * BLOCK + threadIdx.x;
    if (c >= S.k) return;
    const int total = S.cnbr_start[S.k];
    if (c == 0) S.sc->cnbr_total = total;
    if (total > S.cnbr_cap || (S.sc->err & ERR_CNBR)) {
        if (c == 0) atomicOr(&S.sc->err, ERR_CNBR);
        return;
    }
    const int b = S.cnbr_start[c];
    (void)cell_query_serial(S, S.sc, c, search, 1, S.cnbr + b, S.cnbr_start[c + 1] - b);
}

__global__ __launch_bounds__(BLOCK) void k_cnbr_count(const SysDev *Sd, Maps L_maps, double search) {
    const int cbk = blockIdx.x / CQ_BLOCKS;
    if (cbk >= L_maps.c[L_maps.nsys]) return;
    const int s = find_sys(L_maps.c, L_maps.nsys, cbk);
    const SysDev &S = Sd[s];
    if (!S.sc->rebuild || S.k >= CQ_SERIAL_MIN) return;
    const int lb = cbk - L_maps.c[s];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const int c0 = lb * BLOCK + ((blockIdx.x % CQ_BLOCKS) * (BLOCK / WAVE) + wv) * CQ_WAVE;
    int m = 0;
    for (int k = 0; k < CQ_WAVE; ++k) {
        const int c = c0 + k;
        if (c >= S.k) break;                       // wavefront-uniform
        int n = cell_query_wave(S, S.sc, c, search, nullptr, 0);
        if (n > CNBR_ROW_MAX) {                    // keeps the scanned total inside int32
            if (lane == 0) atomicOr(&S.sc->err, ERR_CNBR);
            n = 0;
        }
        if (lane == 0) S.cnbr_start[c] = n;
        m = max(m, n);
    }
    __shared__ int s_m[BLOCK / WAVE];
    if (lane == 0) s_m[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int mm = max(max(s_m[0], s_m[1]), max(s_m[2], s_m[3]));
        if (mm > 0) max_if_larger(&S.sc->cnbr_maxrow, mm);
    }
}

__global__ __launch_bounds__(BLOCK) void k_cnbr_fill(const SysDev *Sd, Maps L_maps, double search) {
    const int cbk = blockIdx.x / CQ_BLOCKS;
    if (cbk >= L_maps.c[L_maps.nsys]) return;
    const int s = find_sys(L_maps.c, L_maps.nsys, cbk);
    const SysDev &S = Sd[s];
    if (!S.sc->rebuild || S.k >= CQ_SERIAL_MIN) return;
    const int lb = cbk - L_maps.c[s];
    const int wv = threadIdx.x / WAVE;
    const bool first = lb == 0 && blockIdx.x % CQ_BLOCKS == 0 && threadIdx.x == 0;
    const int total = S.cnbr_start[S.k];
    if (first) S.sc->cnbr_total = total;
    if (total > S.cnbr_cap || (S.sc->err & ERR_CNBR)) {
        if (first) atomicOr(&S.sc->err, ERR_CNBR);
        return;
    }
    const int c0 = lb * BLOCK + ((blockIdx.x % CQ_BLOCKS) * (BLOCK / WAVE) + wv) * CQ_WAVE;
    for (int k = 0; k < CQ_WAVE; ++k) {
        const int c = c0 + k;
        if (c >= S.k) break;
        const int b = S.cnbr_start[c];
        const int room = S.cnbr_start[c + 1] - b;
        (void)cell_query_wave(S, S.sc, c, search, S.cnbr + b, room);
    }
}

void launch_cell_bounds(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_cell_bounds, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

void launch_cell_pairs(const LaunchCtx &L) {
    if (L.nblk_c == 0) return;
    // each size class's kernels only where the launch holds a system of that class
    const bool large = L.kmax >= CQ_SERIAL_MIN, small = L.kmin < CQ_SERIAL_MIN;
    if (large)
        hipLaunchKernelGGL(k_cnbr_count_serial, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm.cell_search);
    if (small)
        hipLaunchKernelGGL(k_cnbr_count, dim3(CQ_BLOCKS * L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps,
                           L.prm.cell_search);
    launch_scan(L, 3);
    if (large)
        hipLaunchKernelGGL(k_cnbr_fill_serial, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm.cell_search);
    if (small)
        hipLaunchKernelGGL(k_cnbr_fill, dim3(CQ_BLOCKS * L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps,
                           L.prm.cell_search);
}

// ------------------------------------------------------------------ neighbour lists

// In-place exclusive scan of a[0..n), n <= 8 * BLOCK, by the whole block; returns the total.
__device__ int block_scan_lds(int *a, int n, int *s_w) {
    int v[8];
    int loc = 0;
    const int base = threadIdx.x * 8;
    for (int q = 0; q < 8; ++q) {
        const int idx = base + q;
        v[q] = idx < n ? a[idx] : 0;
        loc += v[q];
    }
    int tot;
    int ex = block_excl_scan(loc, s_w, tot);
    for (int q = 0; q < 8; ++q) {
        const int idx = base + q;
        if (idx < n) a[idx] = ex;
        ex += v[q];
    }
    __syncthreads();
    return tot;
}

__device__ __forceinline__ int lds_lower_bound(const int *a, int n, int v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int m = (lo + hi) >> 1;
        if (a[m] < v) lo = m + 1; else hi = m;
    }
    return lo;
}

// One of three FP32 radii by partner type, as integer selects (no branches).
__device__ __forceinline__ float sel3f(int t, float a, float b, float c) {
    int r = (t == 1) ? __float_as_int(b) : __float_as_int(c);
    r = (t == 0) ? __float_as_int(a) : r;
    return __int_as_float(r);
}

// 32 byte flags (each 0 or 1, 4-byte aligned in LDS) as one word, flag k in bit k.
// Marking set members with plain byte stores of 1 avoids serialising many lanes'
// atomics on a few bitmap words.
__device__ __forceinline__ unsigned pack_flags(const unsigned char *f) {
    const unsigned *w = reinterpret_cast<const unsigned *>(f);
    unsigned bits = 0u;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const unsigned v = w[q];
        bits |= ((v & 1u) | ((v >> 7) & 2u) | ((v >> 14) & 4u) | ((v >> 21) & 8u)) << (4 * q);
    }
    return bits;
}

// Last candidate cell whose particle offset is <= u (offsets of empty cells repeat).
__device__ __forceinline__ int union_cell(const int *ofs, int nsc, int u) {
    int lo = 0, hi = nsc;
    while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (ofs[m] <= u) lo = m; else hi = m;
    }
    return lo;
}

// Smallest and largest coordinates of each wavefront's particles (FP32 offsets;
// lanes without a particle pass +inf and -inf), in s_b[6 w .. 6 w + 5].
__device__ __forceinline__ void chunk_box(const float lo_in[3], const float hi_in[3], float *s_b) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float mn[3] = {lo_in[0], lo_in[1], lo_in[2]}, mx[3] = {hi_in[0], hi_in[1], hi_in[2]};
    for (int off = 32; off > 0; off >>= 1)
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], __shfl_xor(mn[a], off));
            mx[a] = fmaxf(mx[a], __shfl_xor(mx[a], off));
        }
    if (lane == 0)
        for (int a = 0; a < 3; ++a) {
            s_b[w * 6 + a] = mn[a];
            s_b[w * 6 + 3 + a] = mx[a];
        }
}

// One block per 256 consecutive cell-sorted particles (four 64-particle chunks).
// Candidates: the cell-pair entries of the block's (consecutive) cells, sorted and
// deduplicated in LDS; their particles, in cell order, form the block's candidate
// union.  The union's particles within the largest list radius of the bounding box of
// the block's own particles form the block's stage (a superset of its partners), held
// in LDS as FP32 offsets from the block's first particle with slot and type packed in
// w, cell by cell.  Each lane then collects every partner within the list radius (rc +
// 2 skin of the pair's types) by scanning the staged particles of the cells paired
// with its own cell, after culling each cell by its bounding sphere.  The test runs in
// FP32 against the list radius widened by 1e-3 sigma, which bounds the offsets'
// rounding (offsets are limited to 4096 sigma), so the list is a superset of the FP64
// one; the step kernel decides every pair exactly.  The 16-bit lists hold stage
// indices (0xffff pads), in candidate order.  Blocks whose stage does not fit keep
// 32-bit lists of global slots (stage count -1), built on FP64 positions.
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(1, 3))) void k_nlist(const SysDev *Sd, Maps L_maps, DevParams P) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    __shared__ int s_cand[CANDMAX];
    __shared__ int s_ofs[CANDMAX + 1];
    static_assert(CANDBITS / 32 <= CANDMAX, "the candidate bitmap and its prefix counts overlay s_ofs and s_kofs");
    __shared__ int s_kofs[CANDMAX + 1];
    __shared__ int s_qpos[CANDMAX];
    __shared__ F4 s_u[USTAGE];
    __shared__ F4 s_cb[CULLMAX];
    __shared__ float s_b[24];
    __shared__ int s_w[16];
    __shared__ int s_rows, s_big;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int chunk = lb * (BLOCK / WAVE) + wv;
    const bool chunk_ok = chunk < S.nchunk;
    const int i = lb * BLOCK + tid;
    const bool valid = i < S.n;
    if (S.sc->err & ERR_CNBR) {          // no valid cell pairs: publish empty lists (block-uniform)
        if (lane == 0 && chunk_ok) { S.nlk[chunk] = 0; S.ilk[chunk] = 0; }
        if (tid == 0) { S.scount[lb] = 0; S.iscount[lb] = 0; }
        return;
    }
    if (tid == 0) { s_rows = 0; s_big = 0; }
    // ---- candidate cells, their particle offsets, and the union position of every cell-pair entry
    const int first = lb * BLOCK;
    const int last = min(S.n - 1, first + BLOCK - 1);
    const int c0 = S.owner[first], c1 = S.owner[last];
    const int q0 = S.cnbr_start[c0];
    const int ncand = S.cnbr_start[c1 + 1] - q0;
    const bool have_union = !(ncand <= 0 || ncand > CANDMAX || c1 < c0);
    int nsc = 0, ss = 0;
    if (have_union) {
        // the range of the candidate cell ids: where it spans at most CANDBITS ids, a
        // bitmap over it (in s_ofs, with the words' prefix counts in s_kofs, both free
        // until the stage) sorts and deduplicates them; otherwise a bitonic sort does
        int mn = INT_MAX, mx = INT_MIN;
        for (int q = tid; q < ncand; q += BLOCK) {
            const int v = ldg(S.cnbr + q0 + q);
            mn = min(mn, v);
            mx = max(mx, v);
        }
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, __shfl_xor(mn, o));
            mx = max(mx, __shfl_xor(mx, o));
        }
        if (lane == 0) { s_w[wv] = mn; s_w[8 + wv] = mx; }
        __syncthreads();
        mn = min(min(s_w[0], s_w[1]), min(s_w[2], s_w[3]));
        mx = max(max(s_w[8], s_w[9]), max(s_w[10], s_w[11]));
        __syncthreads();
        if (mx - mn < CANDBITS) {
            unsigned *bm = reinterpret_cast<unsigned *>(s_ofs);
            int *wpre = s_kofs;
            const int nw = ((mx - mn) >> 5) + 1;
            for (int w = tid; w < nw; w += BLOCK) bm[w] = 0u;
            __syncthreads();
            for (int q = tid; q < ncand; q += BLOCK) {
                const int v = ldg(S.cnbr + q0 + q) - mn;
                atomicOr(&bm[v >> 5], 1u << (v & 31));
            }
            __syncthreads();
            for (int w = tid; w < nw; w += BLOCK) wpre[w] = __popc(bm[w]);
            __syncthreads();
            nsc = block_scan_lds(wpre, nw, s_w);
            for (int w = tid; w < nw; w += BLOCK) {
                unsigned b = bm[w];
                int r = wpre[w];
                while (b) {
                    s_cand[r++] = mn + (w << 5) + (__ffs(b) - 1);
                    b &= b - 1u;
                }
            }
            for (int q = tid; q < ncand; q += BLOCK) {
                const int v = ldg(S.cnbr + q0 + q) - mn;
                s_qpos[q] = wpre[v >> 5] + __popc(bm[v >> 5] & ((1u << (v & 31)) - 1u));
            }
            __syncthreads();
            for (int q = tid; q < nsc; q += BLOCK) s_ofs[q] = ldg(S.ccount + s_cand[q]);
        } else {
            int pw = 1;
            while (pw < ncand) pw <<= 1;
            for (int q = tid; q < pw; q += BLOCK) s_cand[q] = (q < ncand) ? ldg(S.cnbr + q0 + q) : INT_MAX;
            __syncthreads();
            for (int kk = 2; kk <= pw; kk <<= 1)
                for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                    for (int t = tid; t < pw; t += BLOCK) {
                        int ixj = t ^ jj;
                        if (ixj > t) {
                            int va = s_cand[t], vb = s_cand[ixj];
                            bool up = (t & kk) == 0;
                            if ((va > vb) == up) { s_cand[t] = vb; s_cand[ixj] = va; }
                        }
                    }
                    __syncthreads();
                }
            // deduplicate in place
            int vals[CANDMAX / BLOCK], fl[CANDMAX / BLOCK], loc = 0;
            for (int q = 0; q < CANDMAX / BLOCK; ++q) {
                const int idx = tid * (CANDMAX / BLOCK) + q;
                vals[q] = idx < pw ? s_cand[idx] : INT_MAX;
                const int prev = (idx > 0 && idx < pw) ? s_cand[idx - 1] : INT_MIN;
                fl[q] = (idx < ncand && (idx == 0 || vals[q] != prev)) ? 1 : 0;
                loc += fl[q];
            }
            int p = block_excl_scan(loc, s_w, nsc);
            for (int q = 0; q < CANDMAX / BLOCK; ++q)
                if (fl[q]) s_cand[p++] = vals[q];
            __syncthreads();
            for (int q = tid; q < nsc; q += BLOCK) s_ofs[q] = ldg(S.ccount + s_cand[q]);
            for (int q = tid; q < ncand; q += BLOCK) s_qpos[q] = lds_lower_bound(s_cand, nsc, ldg(S.cnbr + q0 + q));
        }
        __syncthreads();
        ss = block_scan_lds(s_ofs, nsc, s_w);
        if (tid == 0) s_ofs[nsc] = ss;
        __syncthreads();
    }
    // ---- the stage: the union's particles near the block, as FP32 offsets, cell by
    // cell (s_kofs: each candidate cell's first stage entry), with the candidate cells'
    // centroids and radii (widened by 2e-3 sigma for the offsets' rounding)
    const bool cull = nsc <= CULLMAX;
    const D4 ref = ld3(S.pos + first);
    const D4 pi = valid ? ldpos(S, i) : ref;
    float oi[3] = {(float)minimg1(pi.x - ref.x, S.per[0], S.box[0]), (float)minimg1(pi.y - ref.y, S.per[1], S.box[1]),
                   (float)minimg1(pi.z - ref.z, S.per[2], S.box[2])};
    if (!valid) oi[0] = oi[1] = oi[2] = 0.0f;
    int kept = 0;
    // offsets beyond LIST_EXTENT (or not finite) leave the block without a stage
    auto far = [](const float o[3]) {
        return !(fabsf(o[0]) <= LIST_EXTENT && fabsf(o[1]) <= LIST_EXTENT && fabsf(o[2]) <= LIST_EXTENT);
    };
    if (have_union) {
        if (cull)
            for (int q = tid; q < nsc; q += BLOCK) {
                const D4 c = ldg(S.seed + s_cand[q]);
                const float ox = (float)minimg1(c.x - ref.x, S.per[0], S.box[0]);
                const float oy = (float)minimg1(c.y - ref.y, S.per[1], S.box[1]);
                const float oz = (float)minimg1(c.z - ref.z, S.per[2], S.box[2]);
                s_cb[q] = F4{ox, oy, oz, (float)c.w + 2e-3f};
                const float o[3] = {ox, oy, oz};
                if (far(o)) s_big = 1;
            }
        // the boxes of the block's four chunks, widened by the largest list radius (plus
        // 1e-3 for the rounding of the distance to them): a particle farther from every
        // box has no partner in the block.  A periodic axis measures the distance to a
        // box's centre by the minimum image, and keeps every particle where the widened
        // box spans a quarter of the period or more.  A chunk without particles has no box.
        {
            const float lo_in[3] = {valid ? oi[0] : INFINITY, valid ? oi[1] : INFINITY, valid ? oi[2] : INFINITY};
            const float hi_in[3] = {valid ? oi[0] : -INFINITY, valid ? oi[1] : -INFINITY, valid ? oi[2] : -INFINITY};
            chunk_box(lo_in, hi_in, s_b);
        }
        __syncthreads();
        const float rb = fmaxf(P.rlmaxf[0], fmaxf(P.rlmaxf[1], P.rlmaxf[2])) + 1e-3f;
        constexpr int NB = BLOCK / WAVE;
        float bc[NB][3], bw[NB][3], L[3], iL[3];
        for (int a = 0; a < 3; ++a) {
            L[a] = S.per[a] ? (float)S.box[a] : 0.0f;
            iL[a] = S.per[a] ? 1.0f / L[a] : 0.0f;
        }
        for (int w = 0; w < NB; ++w) {
            const bool empty = !(s_b[w * 6] <= s_b[w * 6 + 3]);
            for (int a = 0; a < 3; ++a) {
                const float lo = s_b[w * 6 + a], hi = s_b[w * 6 + 3 + a];
                bc[w][a] = empty ? 0.0f : 0.5f * (lo + hi);
                bw[w][a] = empty ? -INFINITY : 0.5f * (hi - lo) + 1e-3f;   // half width; rounding of bc covered
                if (!empty && S.per[a] && !(4.0f * (bw[w][a] + rb) < L[a])) bw[w][a] = INFINITY;
            }
        }
        for (int u0 = 0; u0 < ss; u0 += BLOCK) {
            const int u = u0 + tid;
            bool keep = false;
            F4 rec = F4{0.0f, 0.0f, 0.0f, 0.0f};
            int c = -1;
            if (u < ss) {
                c = union_cell(s_ofs, nsc + 1, u);
                const int slot = ldg(S.cstart + s_cand[c]) + (u - s_ofs[c]);
                const D4 pj = ldpos(S, slot);
                const float o[3] = {(float)minimg1(pj.x - ref.x, S.per[0], S.box[0]),
                                    (float)minimg1(pj.y - ref.y, S.per[1], S.box[1]),
                                    (float)minimg1(pj.z - ref.z, S.per[2], S.box[2])};
                if (far(o)) s_big = 1;
                float e2min = INFINITY;
                for (int w = 0; w < NB; ++w) {
                    float e2 = 0.0f;
                    for (int a = 0; a < 3; ++a) {
                        float d = o[a] - bc[w][a];
                        if (S.per[a]) d -= L[a] * rintf(d * iL[a]);
                        const float e = bw[w][a] == INFINITY ? 0.0f : fmaxf(fabsf(d) - bw[w][a], 0.0f);
                        e2 += e * e;
                    }
                    e2min = fminf(e2min, e2);
                }
                keep = e2min <= rb * rb;
                rec = F4{o[0], o[1], o[2], __int_as_float((slot << 2) | ((int)pj.w & 3))};
            }
            int tot;
            const int k = kept + block_excl_scan(keep ? 1 : 0, s_w, tot);
            if (keep && k < USTAGE) s_u[k] = rec;
            // each cell's first stage entry (cells without particles share the next one's)
            if (u < ss && u == s_ofs[c])
                for (int c2 = c; c2 >= 0 && s_ofs[c2] == u; --c2) s_kofs[c2] = k;
            kept += tot;
        }
        for (int c = tid; c <= nsc; c += BLOCK)
            if (s_ofs[c] == ss) s_kofs[c] = kept;
        __syncthreads();
    }
    const bool staged = have_union && kept <= USTAGE && s_big == 0;
    // ---- the lists, and the pruned lists (partners within rc + 2 inner skin) with the
    // stage entries they use flagged in s_pflag (the candidate cells are done with)
    unsigned char *s_pflag = reinterpret_cast<unsigned char *>(s_cand);
    static_assert(sizeof(s_cand) >= USTAGE, "pruned-stage flags overlay the candidate cells");
    for (int w = tid; w < USTAGE / 4; w += BLOCK) reinterpret_cast<unsigned *>(s_pflag)[w] = 0u;
    __syncthreads();
    int cnt = 0, pc = 0;
    int32_t *col = S.nl + (size_t)(chunk_ok ? chunk : 0) * MAXNB * CHUNK + lane;
    uint16_t *col16 = S.nl16 + (size_t)(chunk_ok ? chunk : 0) * MAXNB * CHUNK + lane;
    uint16_t *icol = S.il16 + (size_t)(chunk_ok ? chunk : 0) * MAXNB * CHUNK + lane;
    if (valid && staged) {
        const int ti = (int)pi.w;
        const int A = S.owner[i];
        const float oix = oi[0], oiy = oi[1], oiz = oi[2];
        const float rlA = P.rl2f[ti][0], rlB = P.rl2f[ti][1], rlC = P.rl2f[ti][2];
        const float riA = P.rin2f[ti][0], riB = P.rin2f[ti][1], riC = P.rin2f[ti][2];
        const float rlmax = P.rlmaxf[ti];
        const int selfw = (i << 2) | (ti & 3);            // this particle's own stage record
        const bool periodic = (S.per[0] | S.per[1] | S.per[2]) != 0;
        const float Lx = S.per[0] ? (float)S.box[0] : 0.0f, Ly = S.per[1] ? (float)S.box[1] : 0.0f,
                    Lz = S.per[2] ? (float)S.box[2] : 0.0f;
        const float iLx = S.per[0] ? 1.0f / Lx : 0.0f, iLy = S.per[1] ? 1.0f / Ly : 0.0f,
                    iLz = S.per[2] ? 1.0f / Lz : 0.0f;
        const int qa = S.cnbr_start[A] - q0, qb = S.cnbr_start[A + 1] - q0;
        auto scan_cells = [&](auto per_tag) {
            constexpr bool PER = decltype(per_tag)::value;
            for (int q = qa; q < qb; ++q) {
                const int pos = s_qpos[q];
                if (cull) {
                    // skip cells whose bounding sphere lies beyond the list radius
                    const F4 cb = s_cb[pos];
                    float dx = cb.x - oix, dy = cb.y - oiy, dz = cb.z - oiz;
                    if constexpr (PER) {
                        dx -= Lx * rintf(dx * iLx);
                        dy -= Ly * rintf(dy * iLy);
                        dz -= Lz * rintf(dz * iLz);
                    }
                    const float rr = cb.w + rlmax;
                    if (dx * dx + dy * dy + dz * dz > rr * rr) continue;
                }
                const int ke = s_kofs[pos + 1];
                auto test = [&](const F4 &c, int k) {
                    float dx = c.x - oix, dy = c.y - oiy, dz = c.z - oiz;
                    if constexpr (PER) {
                        dx -= Lx * rintf(dx * iLx);
                        dy -= Ly * rintf(dy * iLy);
                        dz -= Lz * rintf(dz * iLz);
                    }
                    const float d2 = dx * dx + dy * dy + dz * dz;
                    const int w = __float_as_int(c.w);
                    const float rl = sel3f(w & 3, rlA, rlB, rlC);
                    if (d2 < rl && w != selfw) {
                        if (cnt < MAXNB) {
                            stg(col16 + cnt * CHUNK, (uint16_t)k);
                            // the pruned list: the entries within the pruned radius
                            if (d2 < sel3f(w & 3, riA, riB, riC)) {
                                stg(icol + pc * CHUNK, (uint16_t)k);
                                ++pc;
                                s_pflag[k] = 1;
                            }
                        }
                        ++cnt;
                    }
                };
                int k = s_kofs[pos];
                for (; k + 3 < ke; k += 4) {                      // four candidates per trip
                    const F4 a0 = s_u[k], a1 = s_u[k + 1], a2 = s_u[k + 2], a3 = s_u[k + 3];
                    test(a0, k);
                    test(a1, k + 1);
                    test(a2, k + 2);
                    test(a3, k + 3);
                }
                for (; k < ke; ++k) test(s_u[k], k);
            }
        };
        if (periodic) scan_cells(std::true_type{});
        else scan_cells(std::false_type{});
    } else if (valid) {
        const int ti = (int)pi.w;
        const int A = S.owner[i];
        for (int q = S.cnbr_start[A]; q < S.cnbr_start[A + 1]; ++q) {
            int B = ldg(S.cnbr + q);
            int b = ldg(S.cstart + B), e = b + ldg(S.ccount + B);
            for (int j = b; j < e; ++j) {
                if (j == i) continue;
                D4 pj = ldpos(S, j);
                double dx, dy, dz;
                double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
                if (d2 < P.rl2[ti][(int)pj.w]) {
                    if (cnt < MAXNB) stg(col + cnt * CHUNK, (int32_t)j);
                    ++cnt;
                }
            }
        }
    }
    int rows = wave_max_int(cnt);
    if (rows > MAXNB) {
        if (lane == 0) atomicOr(&S.sc->err, ERR_NLIST);
        rows = MAXNB;
    }
    if (chunk_ok && lane == 0) S.nlk[chunk] = rows;
    if (lane == 0) atomicMax(&s_rows, rows);
    // pad every lane to the chunk's row count, and write the stage's slots
    if (chunk_ok) {
        const int mycnt = valid ? min(cnt, MAXNB) : 0;
        if (staged)
            for (int r = mycnt; r < rows; ++r) stg(col16 + r * CHUNK, (uint16_t)0xffff);
        else
            for (int r = mycnt; r < rows; ++r) stg(col + r * CHUNK, (int32_t)-1);
    }
    if (staged)
        for (int k = tid; k < kept; k += BLOCK) stg(S.stage + (size_t)lb * SSTRIDE + k, __float_as_int(s_u[k].w) >> 2);
    // the pruned stage: the flagged stage entries, in stage order; the pruned lists are
    // rewritten as indices into it (each lane reads back what it wrote) and padded to
    // the chunk's row count rounded up to even (the step kernel takes rows in pairs).
    // A block without a stage walks its 32-bit lists unpruned.
    int irows = wave_max_int(min(pc, MAXNB));
    if (!staged) irows = rows;
    if (chunk_ok && lane == 0) S.ilk[chunk] = irows;
    __syncthreads();
    unsigned *s_bits = reinterpret_cast<unsigned *>(s_ofs);          // the union offsets are done with
    int *s_pre = s_ofs + USTAGE / 32;
    static_assert(sizeof(s_ofs) >= 2 * (USTAGE / 32) * sizeof(int), "pruned-stage words overlay the union offsets");
    int nkept = -1;
    if (staged) {
        const int nwords = (kept + 31) / 32;
        for (int w = tid; w < nwords; w += BLOCK) {
            s_bits[w] = pack_flags(s_pflag + 32 * w);
            s_pre[w] = __popc(s_bits[w]);
        }
        __syncthreads();
        nkept = block_scan_lds(s_pre, nwords, s_w);
        for (int k = tid; k < kept; k += BLOCK) {
            const int w = k >> 5;
            const unsigned m = 1u << (k & 31);
            if (s_bits[w] & m)
                stg(S.istage + (size_t)lb * SSTRIDE + s_pre[w] + __popc(s_bits[w] & (m - 1u)), __float_as_int(s_u[k].w) >> 2);
        }
        const int prows = (irows + 1) & ~1;
        const int mine = valid ? min(pc, MAXNB) : 0;
        if (chunk_ok)
            for (int r0 = 0; r0 < prows; r0 += 8) {
                int e[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) e[q] = r0 + q < mine ? (int)ldg(icol + (r0 + q) * CHUNK) : -1;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (r0 + q >= prows) break;
                    int local = 0xffff;
                    if (e[q] >= 0) {
                        const int w = e[q] >> 5;
                        local = s_pre[w] + __popc(s_bits[w] & ((1u << (e[q] & 31)) - 1u));
                    }
                    stg(icol + (r0 + q) * CHUNK, (uint16_t)local);
                }
            }
    }
    __syncthreads();
    if (tid == 0) {
        S.scount[lb] = staged ? kept : -1;
        S.iscount[lb] = nkept;
        if (s_rows > 0) max_if_larger(&S.sc->nlrows, s_rows);   // the build's longest list
    }
}

void launch_nlist(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_nlist, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm);
}

// ------------------------------------------------------------------ pruned lists

// One block per 256 consecutive cell-sorted particles.  The block's lists hold every
// partner within rc + 2 skin at the last build; the partners within rc + 2 inner skin
// are kept in a pruned list, which the force kernel walks instead.  The build writes
// the pruned lists for its own positions; this kernel prunes again between builds, at
// the current positions.  A pair left out was farther apart than rc + 2 inner
// skin when the lists were pruned, so it cannot come within rc before some particle
// has moved more than the inner skin since then; the runtime prunes again before
// that.  As in the list build, the test runs on FP32 offsets from the block's first
// particle against the radius widened by 1e-3 sigma (offsets are limited to 4096
// sigma), so the pruned list is a superset of the exact neighbour set; blocks whose
// offsets exceed that keep every entry.  The partners kept form the block's pruned
// stage (in stage order); the pruned list holds indices into it, padded with 0xffff.
// Blocks without a stage (32-bit global lists) are not pruned (pruned count -1).
// Every particle's current position becomes its reference for the displacement
// since the prune.
__global__ __launch_bounds__(BLOCK) void k_prune(const SysDev *Sd, Maps L_maps, DevParams P) {
    SYS_FROM(p);
    // stage offsets, 12 B each: the type rides in the two low mantissa bits of x (a
    // change of at most three ulp, far inside the 1e-3 sigma widening of the radius)
    __shared__ F3 s_o[SMAX];
    __shared__ __align__(16) unsigned char s_flag[SMAX];   // stage entry kept by some lane (plain stores of 1)
    __shared__ unsigned s_bits[SMAX / 32];
    __shared__ int s_pre[SMAX / 32];
    __shared__ int s_w[16];
    __shared__ int s_big;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int chunk = lb * (BLOCK / WAVE) + wv;
    const bool chunk_ok = chunk < S.nchunk;
    const int i = lb * BLOCK + tid;
    const bool valid = i < S.n;
    if (lb == 0 && tid == 0) S.sc->maxdisp2p = 0ull;
    const D4 pi = valid ? ldpos(S, i) : D4{0.0, 0.0, 0.0, 0.0};
    if (valid) S.xp[i] = F3{(float)pi.x, (float)pi.y, (float)pi.z};
    const int scnt = S.scount[lb];
    const int rows = chunk_ok ? min(S.nlk[chunk], MAXNB) : 0;
    if (scnt < 0) {
        if (chunk_ok && lane == 0) S.ilk[chunk] = rows;
        if (tid == 0) S.iscount[lb] = -1;
        return;
    }
    if (tid == 0) s_big = 0;
    for (int w = tid; w < SMAX / 4; w += BLOCK) reinterpret_cast<unsigned *>(s_flag)[w] = 0u;
    const D4 ref = ld3(S.pos + (size_t)lb * BLOCK);
    bool far = false;
    // eight entries per thread in flight: their slots, then their positions
    for (int q0 = tid; q0 < scnt; q0 += 8 * BLOCK) {
        int slot[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = q0 + k * BLOCK;
            slot[k] = q < scnt ? ldg(S.stage + (size_t)lb * SSTRIDE + q) : -1;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int q = q0 + k * BLOCK;
            if (slot[k] < 0) break;
            const D4 pj = ldpos(S, slot[k]);
            const float ox = (float)minimg1(pj.x - ref.x, S.per[0], S.box[0]);
            const float oy = (float)minimg1(pj.y - ref.y, S.per[1], S.box[1]);
            const float oz = (float)minimg1(pj.z - ref.z, S.per[2], S.box[2]);
            s_o[q] = F3{__int_as_float((__float_as_int(ox) & ~3) | ((int)pj.w & 3)), oy, oz};
            far = far || !(fabsf(ox) <= LIST_EXTENT && fabsf(oy) <= LIST_EXTENT && fabsf(oz) <= LIST_EXTENT);
        }
    }
    if (far) s_big = 1;                              // offsets out of range or not finite
    __syncthreads();
    const bool keep_all = s_big != 0;
    int cnt = 0;
    const uint16_t *col = S.nl16 + (size_t)(chunk_ok ? chunk : 0) * MAXNB * CHUNK + lane;
    uint16_t *icol = S.il16 + (size_t)(chunk_ok ? chunk : 0) * MAXNB * CHUNK + lane;
    constexpr int BATCH = 32;    // list rows whose entries are loaded together
    if (valid && chunk_ok) {
        const int ti = (int)pi.w;
        const float oix = (float)minimg1(pi.x - ref.x, S.per[0], S.box[0]);
        const float oiy = (float)minimg1(pi.y - ref.y, S.per[1], S.box[1]);
        const float oiz = (float)minimg1(pi.z - ref.z, S.per[2], S.box[2]);
        const float rA = ti == 0 ? P.rin2f[0][0] : (ti == 1 ? P.rin2f[1][0] : P.rin2f[2][0]);
        const float rB = ti == 0 ? P.rin2f[0][1] : (ti == 1 ? P.rin2f[1][1] : P.rin2f[2][1]);
        const float rC = ti == 0 ? P.rin2f[0][2] : (ti == 1 ? P.rin2f[1][2] : P.rin2f[2][2]);
        const bool periodic = (S.per[0] | S.per[1] | S.per[2]) != 0;
        const float Lx = S.per[0] ? (float)S.box[0] : 0.0f, Ly = S.per[1] ? (float)S.box[1] : 0.0f,
                    Lz = S.per[2] ? (float)S.box[2] : 0.0f;
        const float iLx = S.per[0] ? 1.0f / Lx : 0.0f, iLy = S.per[1] ? 1.0f / Ly : 0.0f,
                    iLz = S.per[2] ? 1.0f / Lz : 0.0f;
        for (int r0 = 0; r0 < rows; r0 += BATCH) {
            int e[BATCH];
#pragma unroll
            for (int q = 0; q < BATCH; ++q) e[q] = (int)ldg(col + min(r0 + q, rows - 1) * CHUNK);
#pragma unroll
            for (int q = 0; q < BATCH; ++q) {
                const int eq = (r0 + q < rows) ? e[q] : 0xffff;
                const F3 c = s_o[eq < scnt ? eq : 0];
                float dx = c.x - oix, dy = c.y - oiy, dz = c.z - oiz;
                if (periodic) {
                    dx -= Lx * rintf(dx * iLx);
                    dy -= Ly * rintf(dy * iLy);
                    dz -= Lz * rintf(dz * iLz);
                }
                const float d2 = dx * dx + dy * dy + dz * dz;
                const float rr = sel3f(__float_as_int(c.x) & 3, rA, rB, rC);
                if (eq < scnt && (keep_all || d2 < rr)) {
                    stg(icol + cnt * CHUNK, (uint16_t)eq);
                    ++cnt;
                    s_flag[eq] = 1;
                }
            }
        }
    }
    const int irows = wave_max_int(cnt);
    if (chunk_ok && lane == 0) S.ilk[chunk] = irows;
    __syncthreads();
    const int nwords = (scnt + 31) / 32;
    for (int w = tid; w < nwords; w += BLOCK) {
        s_bits[w] = pack_flags(s_flag + 32 * w);
        s_pre[w] = __popc(s_bits[w]);
    }
    __syncthreads();
    const int nkept = block_scan_lds(s_pre, nwords, s_w);
    // the pruned stage: every kept entry's slot at its rank among the kept entries
    for (int q = tid; q < scnt; q += BLOCK) {
        const int w = q >> 5;
        const unsigned m = 1u << (q & 31);
        if (s_bits[w] & m)
            stg(S.istage + (size_t)lb * SSTRIDE + s_pre[w] + __popc(s_bits[w] & (m - 1u)),
                ldg(S.stage + (size_t)lb * SSTRIDE + q));
    }
    // rewrite the kept entries as pruned-stage indices (the lane reads back what it
    // wrote), padding every lane to the chunk's row count rounded up to even (the step
    // kernel takes rows in pairs)
    const int prows = (irows + 1) & ~1;
    if (chunk_ok)
        for (int r0 = 0; r0 < prows; r0 += BATCH) {
            int e[BATCH];
#pragma unroll
            for (int q = 0; q < BATCH; ++q) e[q] = r0 + q < cnt ? (int)ldg(icol + (r0 + q) * CHUNK) : -1;
#pragma unroll
            for (int q = 0; q < BATCH; ++q) {
                if (r0 + q >= prows) break;
                int local = 0xffff;
                if (e[q] >= 0) {
                    const int w = e[q] >> 5;
                    local = s_pre[w] + __popc(s_bits[w] & ((1u << (e[q] & 31)) - 1u));
                }
                stg(icol + (r0 + q) * CHUNK, (uint16_t)local);
            }
        }
    if (tid == 0) S.iscount[lb] = nkept;
}

// Block map of the systems in the mask (particle blocks only), for prunes outside a
// cell update.  One block of MAX_SLOTS threads.
__global__ __launch_bounds__(MAX_SLOTS) void k_mask_maps(const SysDev *Sd, int nsys, unsigned long long m0,
                                                         unsigned long long m1, unsigned long long m2,
                                                         unsigned long long m3, int32_t *out) {
    __shared__ int s_w[16];
    const int s = threadIdx.x;
    int cnt = 0;
    if (s < nsys) {
        const unsigned long long w = (s < 64) ? m0 : (s < 128) ? m1 : (s < 192) ? m2 : m3;
        if ((w >> (s & 63)) & 1ull) cnt = (Sd[s].n + BLOCK - 1) / BLOCK;
    }
    int tot;
    const int ex = block_excl_scan(cnt, s_w, tot);
    if (s <= nsys) out[s] = ex;
}

void launch_prune(const LaunchCtx &L) {
    if (L.nblk_p > 0) hipLaunchKernelGGL(k_prune, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm);
}

void launch_mask_maps(const LaunchCtx &L, const unsigned long long m[4], int32_t *out) {
    hipLaunchKernelGGL(k_mask_maps, dim3(1), dim3(MAX_SLOTS), 0, L.st, L.S, L.nsys, m[0], m[1], m[2], m[3], out);
}

// ------------------------------------------------------------------ finish

// The drift references of the new lists, and after a cell update (the particles have
// moved to new slots) the FP32 orientation copies; between updates the step kernel
// keeps those current.
__global__ void k_finish_particles(const SysDev *Sd, Maps L_maps, int cells_moved) {
    SYS_FROM(p);
    if (!S.sc->rebuild) return;
    int i = lb * BLOCK + threadIdx.x;
    if (i < S.n) {
        const V3 p = S.pos[i];
        S.xb[i] = F3{(float)p.x, (float)p.y, (float)p.z};
        S.xp[i] = F3{(float)p.x, (float)p.y, (float)p.z};
        if (cells_moved) {
            const V3 o = S.ori[i];
            S.ori32[i] = F4{(float)o.x, (float)o.y, (float)o.z, __int_as_float((int)S.typ[i] & TYP_MASK)};
        }
    }
}

__global__ __launch_bounds__(256) void k_finish_sys(const SysDev *Sd, int nsys) {
    const SysDev &S = Sd[blockIdx.x];
    SysScal *sc = S.sc;
    if (!sc->rebuild) return;
    if (threadIdx.x == 0) {
        sc->maxdisp2 = 0ull;
        sc->maxv2 = 0ull;
        sc->maxdisp2p = 0ull;
        sc->rebuild = 0;
    }
}

void launch_finish_update(const LaunchCtx &L, bool cells_moved) {
    hipLaunchKernelGGL(k_finish_particles, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, cells_moved ? 1 : 0);
    hipLaunchKernelGGL(k_finish_sys, dim3(L.nsys), dim3(256), 0, L.st, L.S, L.nsys);
}

// ------------------------------------------------------------------ entry points used by the runtime

// Block maps restricted to the systems that rebuild (the others get no blocks), so
// an update launches only the rebuilding systems' blocks.  The block counts per
// system match the full maps built on the host; one block of MAX_SLOTS threads.
__global__ __launch_bounds__(MAX_SLOTS) void k_restrict_maps(const SysDev *Sd, int nsys, int32_t *out) {
    __shared__ int s_w[16];
    const int s = threadIdx.x;
    int cnt[7] = {0, 0, 0, 0, 0, 0, 0};
    if (s < nsys) {
        const SysDev &S = Sd[s];
        if (S.n > 0 && S.sc->rebuild) {
            cnt[0] = (S.n + BLOCK - 1) / BLOCK;
            cnt[1] = (S.k + BLOCK - 1) / BLOCK;
            cnt[2] = (S.gcap + BLOCK - 1) / BLOCK;
            cnt[3] = S.ntile_p;
            cnt[4] = S.ntile_s;
            cnt[5] = (S.k + SCAN_TILE - 1) / SCAN_TILE;
            cnt[6] = (S.gcap + SCAN_TILE - 1) / SCAN_TILE;
        }
    }
    for (int m = 0; m < 7; ++m) {
        int tot;
        const int ex = block_excl_scan(cnt[m], s_w, tot);
        if (s <= nsys) out[m * (nsys + 1) + s] = ex;     // entry nsys receives the total
    }
}

void launch_restrict_maps(const LaunchCtx &L, int32_t *out) {
    hipLaunchKernelGGL(k_restrict_maps, dim3(1), dim3(MAX_SLOTS), 0, L.st, L.S, L.nsys, out);
}

void launch_set_rebuild(const LaunchCtx &L, const unsigned long long m[4]) {
    hipLaunchKernelGGL(k_set_rebuild, dim3((L.nsys + 63) / 64), dim3(64), 0, L.st, L.S, L.nsys, m[0], m[1], m[2],
                       m[3]);
}

void launch_init_seeds(const LaunchCtx &L, const int32_t *const *lipids) {
    hipLaunchKernelGGL(k_init_seeds, dim3(L.nblk_c), dim3(BLOCK), 0, L.st, L.S, L.maps, lipids);
    hipLaunchKernelGGL(k_clear_owner, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

void launch_pack(const LaunchCtx &L, int s, const double *x, const double *n, const int32_t *type,
                 const double *v, const double *w, int count) {
    hipLaunchKernelGGL(k_pack_multi, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, L.st, L.S, s, x, n, type,
                       v, w);
}

}  // namespace rbc
