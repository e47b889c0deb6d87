// Pair force / torque evaluation and the velocity-Verlet step on gfx950.
//
// Force Evaluation section: pairwise lipid-lipid, lipid-protein and
// protein-protein forces are found through the Voronoi cells (here: the
// per-particle neighbour lists built from the cell pairs at each cell update,
// valid while no particle has moved more than the skin), plus the bonds of
// physically linked proteins.  One wavefront owns a chunk of 64 consecutive
// cell-sorted particles; lane l accumulates the force and torque on particle
// base + l from every partner in column l of the chunk's ELL list, so the
// per-particle sums need no atomics and are bitwise reproducible.  Every
// candidate goes through the exact FP64 neighbour test; the pair law then runs
// in FP64 or, in mixed mode, in FP32 on the FP64-formed separation, while
// energy and virial sums stay FP64.
//
// Software Overview section (time-stepping loop): kick-drift advances positions
// and lipid orientations (free linear-rotor rotation about the angular
// velocity); the second half-kick is fused into the force kernel's epilogue.
#include "rbc_dev.h"

#include <mutex>

namespace rbc {

__device__ __forceinline__ int lane_id_f() { return threadIdx.x & (WAVE - 1); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_maxd(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

template <class T>
__device__ __forceinline__ T ipow(T c, int e) {
    T r = (T)1;
    for (int q = 0; q < e; ++q) r *= c;
    return r;
}

// One of three FP64 cutoffs by partner type, as bit selects (no branches).
__device__ __forceinline__ double sel_cut(int t, double a, double b, double c) {
    long long r = (t == 1) ? __double_as_longlong(b) : __double_as_longlong(c);
    r = (t == 0) ? __double_as_longlong(a) : r;
    return __longlong_as_double(r);
}

__device__ __forceinline__ float sel_cutf(int t, float a, float b, float c) {
    int r = (t == 1) ? __float_as_int(b) : __float_as_int(c);
    r = (t == 0) ? __float_as_int(a) : r;
    return __int_as_float(r);
}

// ------------------------------------------------------------------ pair laws

// Lipid-lipid orientation-dependent law; d = x_i - x_j.  Adds the force and torque
// on i and returns U.  FAST: the default constants zeta = 4 and sin(theta0) = 0
// folded in at compile time (same arithmetic with the zero terms removed).
template <class T, bool FAST>
__device__ __forceinline__ T lipid_pair(const DevParams &P, T dx, T dy, T dz, T nix, T niy, T niz, T njx, T njy,
                                        T njz, T &fx, T &fy, T &fz, T &tx, T &ty, T &tz) {
    const T eps = (T)P.eps, mu = (T)P.mu, st0 = FAST ? (T)0 : (T)P.st0, rmin = (T)P.r_min;
    T r2 = dx * dx + dy * dy + dz * dz;
    T rinv, r;
    if constexpr (sizeof(T) == 4) {
        rinv = __builtin_amdgcn_rsqf(r2);
        r = r2 * rinv;
    } else {
        r = sqrt(r2);
        rinv = (T)1 / r;
    }
    const T ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
    const T s = nix * ex + niy * ey + niz * ez;
    const T t = njx * ex + njy * ey + njz * ez;
    const T c = nix * njx + niy * njy + niz * njz;
    T a = c - s * t;
    if (!FAST) a += st0 * (t - s) - st0 * st0;
    const T phi = (T)1 + mu * (a - (T)1);
    T U, dUdr, dUda;
    if (r < rmin) {
        const T q = (rmin * rinv) * (rmin * rinv);
        U = eps * (q * q - (T)2 * q) + ((T)1 - phi) * eps;
        dUdr = (T)4 * eps * (q - q * q) * rinv;
        dUda = -mu * eps;
    } else {
        T sx, cx;
        const T u = (r - rmin) * (T)P.inv_w;              // (r - r_min) / (r_c - r_min)
        if constexpr (sizeof(T) == 4) {
            // x = (pi/2) u; the hardware sine and cosine take revolutions: x / 2pi = u / 4
            sx = __builtin_amdgcn_sinf((T)0.25 * u);
            cx = __builtin_amdgcn_cosf((T)0.25 * u);
        } else {
            // x = (pi/2) u lies in [0, pi/2): Taylor series of the half angle (terms
            // through h^16; the first omitted one is below 1e-16 relative), then the
            // double-angle formulas
            const double h = 0.25 * M_PI * u, h2 = h * h;
            // nested factors 1 - h^2/(k(k+1)), multiplied by compile-time reciprocals
            const double sh = h * (1.0 - h2 * (1.0 / 6.0) * (1.0 - h2 * (1.0 / 20.0) * (1.0 - h2 * (1.0 / 42.0) *
                              (1.0 - h2 * (1.0 / 72.0) * (1.0 - h2 * (1.0 / 110.0) * (1.0 - h2 * (1.0 / 156.0) *
                              (1.0 - h2 * (1.0 / 210.0))))))));
            const double ch = 1.0 - h2 * 0.5 * (1.0 - h2 * (1.0 / 12.0) * (1.0 - h2 * (1.0 / 30.0) *
                              (1.0 - h2 * (1.0 / 56.0) * (1.0 - h2 * (1.0 / 90.0) * (1.0 - h2 * (1.0 / 132.0) *
                              (1.0 - h2 * (1.0 / 182.0) * (1.0 - h2 * (1.0 / 240.0))))))));
            sx = 2.0 * sh * ch;
            cx = (ch - sh) * (ch + sh);
        }
        const T c2 = cx * cx;
        T cz1;                                            // cos^(2 zeta - 2)
        if (FAST) cz1 = c2 * c2 * c2;
        else cz1 = ipow(c2, P.zeta - 1);
        const T uA = -eps * cz1 * c2;
        U = uA * phi;
        dUdr = phi * (T)P.dudr_k * sx * cz1 * cx;         // phi eps zeta pi / (r_c - r_min) sin x cos^(2 zeta - 1) x
        dUda = mu * uA;
    }
    T gx = -t * nix - s * njx, gy = -t * niy - s * njy, gz = -t * niz - s * njz;
    if (!FAST) {
        gx += st0 * (njx - nix);
        gy += st0 * (njy - niy);
        gz += st0 * (njz - niz);
    }
    const T proj = gx * ex + gy * ey + gz * ez;
    const T k = dUda * rinv;
    fx -= dUdr * ex + k * (gx - proj * ex);
    fy -= dUdr * ey + k * (gy - proj * ey);
    fz -= dUdr * ez + k * (gz - proj * ez);
    // torque on i: n_i x g_i with g_i = -dU/da (n_j - (t + sin th0) e)
    const T bb = t + st0;
    const T wx = -dUda * (njx - bb * ex), wy = -dUda * (njy - bb * ey), wz = -dUda * (njz - bb * ez);
    tx += niy * wz - niz * wy;
    ty += niz * wx - nix * wz;
    tz += nix * wy - niy * wx;
    return U;
}

// WCA for pairs with a protein bead; adds the force on i, returns U.
template <class T>
__device__ __forceinline__ T wca_pair(const DevParams &P, T dx, T dy, T dz, T &fx, T &fy, T &fz) {
    T r2 = dx * dx + dy * dy + dz * dz;
    T r2inv;
    if constexpr (sizeof(T) == 4) r2inv = __builtin_amdgcn_rcpf(r2);
    else r2inv = (T)1 / r2;
    T sr2 = (T)P.wca_sig2 * r2inv;
    T sr6 = sr2 * sr2 * sr2;
    T e = (T)P.wca_eps;
    T U = (T)4 * e * (sr6 * sr6 - sr6) + e;
    T f = (T)24 * e * ((T)2 * sr6 * sr6 - sr6) * r2inv;
    fx += f * dx;
    fy += f * dy;
    fz += f * dz;
    return U;
}

// ------------------------------------------------------------------ integrator pieces

// Free linear-rotor drift: n rotated about omega by |omega| dt (Rodrigues), then
// renormalised.
__device__ __forceinline__ D4 rotor_drift(D4 n, const D4 &w, double dt) {
#pragma clang fp contract(off)
    const double wn = sqrt(w.x * w.x + w.y * w.y + w.z * w.z);
    if (wn > 0.0) {
        const double iw = 1.0 / wn;
        const double kx = w.x * iw, ky = w.y * iw, kz = w.z * iw;
        const double a = wn * dt;
        double sn, cs;
        if (a < 0.05) {
            // Taylor series; the first omitted terms are below 1e-18 relative here
            const double a2 = a * a;
            sn = a * (1.0 - a2 * (1.0 / 6.0) * (1.0 - a2 * (1.0 / 20.0) * (1.0 - a2 * (1.0 / 42.0) *
                 (1.0 - a2 * (1.0 / 72.0)))));
            cs = 1.0 - a2 * 0.5 * (1.0 - a2 * (1.0 / 12.0) * (1.0 - a2 * (1.0 / 30.0) * (1.0 - a2 * (1.0 / 56.0) *
                 (1.0 - a2 * (1.0 / 90.0)))));
        } else {
            sincos(a, &sn, &cs);
        }
        const double kn = kx * n.x + ky * n.y + kz * n.z;
        const double cx = ky * n.z - kz * n.y, cy = kz * n.x - kx * n.z, cz = kx * n.y - ky * n.x;
        const double ox = n.x * cs + cx * sn + kx * kn * (1.0 - cs);
        const double oy = n.y * cs + cy * sn + ky * kn * (1.0 - cs);
        const double oz = n.z * cs + cz * sn + kz * kn * (1.0 - cs);
        n.x = ox; n.y = oy; n.z = oz;
    }
    const double nn = sqrt(n.x * n.x + n.y * n.y + n.z * n.z);
    if (nn > 0.0) {
        const double in = 1.0 / nn;
        n.x *= in; n.y *= in; n.z *= in;
    }
    return n;
}

// Half-kick v += h a, drift x += dt v, and the drift's statistics.  Every
// operation is rounded on its own (no contraction), so the drift fused into the
// force kernel and the standalone kick-drift give the same bits.
__device__ __forceinline__ void half_kick(D4 &v, double h, double ax, double ay, double az) {
#pragma clang fp contract(off)
    v.x += h * ax;
    v.y += h * ay;
    v.z += h * az;
}

__device__ __forceinline__ void drift_pos(D4 &x, const D4 &v, double dt) {
#pragma clang fp contract(off)
    x.x += dt * v.x;
    x.y += dt * v.y;
    x.z += dt * v.z;
}

// Displacements since the last list build and since the last prune, measured
// against FP32 copies of the reference positions (their rounding, below 6e-5 sigma for
// coordinates under 1000 sigma, is covered by the runtime's margins).
__device__ __forceinline__ void drift_measures(const D4 &x, const D4 &v, const F3 &b, const F3 &p, double &disp2,
                                               double &disp2p, double &v2, bool &bad) {
#pragma clang fp contract(off)
    const double ddx = x.x - (double)b.x, ddy = x.y - (double)b.y, ddz = x.z - (double)b.z;
    disp2 = ddx * ddx + ddy * ddy + ddz * ddz;
    const double dpx = x.x - (double)p.x, dpy = x.y - (double)p.y, dpz = x.z - (double)p.z;
    disp2p = dpx * dpx + dpy * dpy + dpz * dpz;
    v2 = v.x * v.x + v.y * v.y + v.z * v.z;
    bad = !isfinite(x.x + x.y + x.z + v.x + v.y + v.z);
}

// The volume's lipid sums of one particle (x.n, x, n, 1; zero for proteins) and
// their per-chunk totals, a fixed butterfly over the wavefront stored
// component-major at vpart[q * nchunk + chunk].  The drift computes them for the
// positions it writes, so the next force evaluation needs only the reduction.
__device__ __forceinline__ void volume_terms(const D4 &x, const D4 &n, double v[8]) {
#pragma clang fp contract(off)
    v[0] = x.x * n.x + x.y * n.y + x.z * n.z;
    v[1] = x.x; v[2] = x.y; v[3] = x.z;
    v[4] = n.x; v[5] = n.y; v[6] = n.z;
    v[7] = 1.0;
}

// Wavefront sum of a double by DPP lane moves in a fixed order (no LDS traffic):
// a Hillis-Steele scan within each 16-lane row (shifts 1, 2, 4, 8), then row 0's
// total into row 1 and row 2's into row 3 (row_bcast:15), then the first half's
// total into rows 2 and 3 (row_bcast:31).  Lane 63 ends with the total.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return v + __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_total_lane63(double v) {
    v = dpp_add<0x111, 0xf>(v);     // row_shr:1
    v = dpp_add<0x112, 0xf>(v);     // row_shr:2
    v = dpp_add<0x114, 0xf>(v);     // row_shr:4
    v = dpp_add<0x118, 0xf>(v);     // row_shr:8
    v = dpp_add<0x142, 0xa>(v);     // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);     // row_bcast:31 into rows 2 and 3
    return v;
}

// The same scan taking maxima, for non-negative values (lanes without a source
// contribute 0).  Lane 63 ends with the largest value.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_max(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return fmax(v, __hiloint2double(hi, lo));
}

__device__ __forceinline__ double wave_max_lane63(double v) {
    v = dpp_max<0x111, 0xf>(v);
    v = dpp_max<0x112, 0xf>(v);
    v = dpp_max<0x114, 0xf>(v);
    v = dpp_max<0x118, 0xf>(v);
    v = dpp_max<0x142, 0xa>(v);
    v = dpp_max<0x143, 0xc>(v);
    return v;
}

__device__ __forceinline__ void volume_chunk_store(const SysDev &S, int chunk, double v[8]) {
    for (int q = 0; q < 8; ++q) v[q] = wave_total_lane63(v[q]);
    if ((threadIdx.x & (WAVE - 1)) == WAVE - 1)
        for (int q = 0; q < 8; ++q) S.vpart[(size_t)q * S.nchunk + chunk] = v[q];
}

// Velocity quenching: keep the part of a along b when it points along b,
// a <- max(a.b, 0) b / |b|^2; and scale a so that |a| dt <= m.  No contraction,
// as for the kicks.
__device__ __forceinline__ void project_along(D4 &a, double bx, double by, double bz) {
#pragma clang fp contract(off)
    const double bb = bx * bx + by * by + bz * bz;
    const double ab = a.x * bx + a.y * by + a.z * bz;
    if (bb > 0.0 && ab > 0.0) {
        const double s = ab / bb;
        a.x = s * bx; a.y = s * by; a.z = s * bz;
    } else {
        a.x = 0.0; a.y = 0.0; a.z = 0.0;
    }
}

__device__ __forceinline__ void cap_move(D4 &a, double dt, double m) {
#pragma clang fp contract(off)
    const double s = sqrt(a.x * a.x + a.y * a.y + a.z * a.z) * dt;
    if (s > m) {
        const double f = m / s;
        a.x *= f; a.y *= f; a.z *= f;
    }
}

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of two 32 x 32
// -> 64-bit products mixed with the other words and the key, which advances by
// the Weyl constants between rounds.
__device__ __forceinline__ void philox10(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Thermostat update of one particle after its closing half-kick: the exact
// Ornstein-Uhlenbeck step v <- c v + sqrt((1 - c^2) kT / m) xi, xi uniform with unit
// variance from the Philox words of counter (caller id, step, 0); lipids also
// w <- c_r w + sqrt((1 - c_r^2) kT / I) (xi' - (xi'.n) n) from counter (.., 1).
// Every operation is rounded on its own (no contraction): the fused and the
// stored-then-reloaded step paths then agree bit for bit.
__device__ __forceinline__ void langevin_update(const DevParams &P, int gid, unsigned long long step, int t,
                                                const D4 &n, D4 &v, D4 &w) {
#pragma clang fp contract(off)
    const uint32_t s_lo = (uint32_t)step, s_hi = (uint32_t)(step >> 32);
    constexpr double half = 2147483647.5;   // (2^32 - 1) / 2: centres the words
    {
        uint32_t c0 = (uint32_t)gid, c1 = s_lo, c2 = s_hi, c3 = 0u;
        philox10(c0, c1, c2, c3, P.seed_lo, P.seed_hi);
        const double a = P.ou_a[t];
        v.x = P.ou_c * v.x + a * ((double)c0 - half);
        v.y = P.ou_c * v.y + a * ((double)c1 - half);
        v.z = P.ou_c * v.z + a * ((double)c2 - half);
    }
    if (t == 0) {
        uint32_t c0 = (uint32_t)gid, c1 = s_lo, c2 = s_hi, c3 = 1u;
        philox10(c0, c1, c2, c3, P.seed_lo, P.seed_hi);
        const double xx = (double)c0 - half, xy = (double)c1 - half, xz = (double)c2 - half;
        const double pn = xx * n.x + xy * n.y + xz * n.z;
        w.x = P.ou_cr * w.x + P.ou_ar * (xx - pn * n.x);
        w.y = P.ou_cr * w.y + P.ou_ar * (xy - pn * n.y);
        w.z = P.ou_cr * w.z + P.ou_ar * (xz - pn * n.z);
    }
}

// Volume term on a lipid: F -= kap (n - nbar), tau += n x (-kap (x - xbar)), each
// operation rounded on its own (the same bits in every kernel variant).
__device__ __forceinline__ void volume_term(const SysScal *sc, const D4 &x, const D4 &n, double &Fx, double &Fy,
                                            double &Fz, D4 &Tq) {
#pragma clang fp contract(off)
    const double kap = sc->volkap;
    Fx -= kap * (n.x - sc->nbar[0]);
    Fy -= kap * (n.y - sc->nbar[1]);
    Fz -= kap * (n.z - sc->nbar[2]);
    const double gx = -kap * (x.x - sc->xbar[0]), gy = -kap * (x.y - sc->xbar[1]), gz = -kap * (x.z - sc->xbar[2]);
    Tq.x += n.y * gz - n.z * gy;
    Tq.y += n.z * gx - n.x * gz;
    Tq.z += n.x * gy - n.y * gx;
}

// Per-wavefront drift statistics: the largest |x - x_build|^2, |v|^2 and
// |x - x_prune|^2 of the wave's particles (chunk w of the particle block) go to the
// block's partial slots 3w, 3w+1 and 3w+2; a non-finite state raises the system's
// error bit.
__device__ __forceinline__ void drift_stats(const SysDev &S, int blk, int w, double &disp2, double &v2, double &disp2p,
                                            bool bad) {
    disp2 = wave_max_lane63(disp2);
    v2 = wave_max_lane63(v2);
    disp2p = wave_max_lane63(disp2p);
    const unsigned long long anybad = __ballot(bad);
    if (lane_id_f() == WAVE - 1) {
        S.bred[(size_t)blk * BRED + 3 * w] = disp2;
        S.bred[(size_t)blk * BRED + 3 * w + 1] = v2;
        S.bred[(size_t)blk * BRED + 3 * w + 2] = disp2p;
        if (anybad) atomicOr(&S.sc->err, ERR_NONFINITE);
    }
}

// The end of a drift's statistics pass over one system, run once by whichever
// block finishes last: the maxima (every block's atomic max is in) go to the host
// ring entry of this drift number, tag last, and the drift is counted.
__device__ __forceinline__ void publish_drift(SysScal *sc, StepStat *hstat) {
    const unsigned long long st = sc->step;
    const unsigned long long d = atomicOr(&sc->maxdisp2, 0ull);
    const unsigned long long v = atomicOr(&sc->maxv2, 0ull);
    const unsigned long long dp = atomicOr(&sc->maxdisp2p, 0ull);
    StepStat *e = hstat + st % STAT_RING;
    e->d2 = bitsd(d);
    e->v2 = bitsd(v);
    e->d2p = bitsd(dp);
    __threadfence_system();
    e->tag = st + 1;
    sc->step = st + 1;
}

__device__ __forceinline__ void swap_drift(SysDev &W);

// A small (split) system publishes its drift statistics from the step kernel itself:
// lane 63 of each workgroup's wave 0 (which holds the wave's maxima after drift_stats)
// folds them into the system's running maxima; the last of the system's nwg
// workgroups (one per chunk) to finish publishes them and swaps the drift buffers, as the statistics
// kernel does for larger systems.  Atomic maxima of non-negative doubles' bit patterns
// do not depend on their order.
__device__ __forceinline__ void publish_split(SysDev &W, int nwg, double disp2, double v2, double disp2p) {
    if (lane_id_f() != WAVE - 1) return;
    SysScal *sc = W.sc;
    atomicMax(&sc->maxdisp2, dbits(disp2));
    atomicMax(&sc->maxv2, dbits(v2));
    atomicMax(&sc->maxdisp2p, dbits(disp2p));
    __threadfence();
    if (atomicAdd(&sc->parts_done, 1u) == (unsigned)nwg - 1u) {
        __threadfence();
        publish_drift(sc, W.hstat);
        sc->parts_done = 0;
        swap_drift(W);
    }
}

__device__ __forceinline__ void swap_drift(SysDev &W) {
    V3 *u = W.pos; W.pos = W.pos2; W.pos2 = u;
    u = W.ori; W.ori = W.ori2; W.ori2 = u;
    F4 *f = W.ori32; W.ori32 = W.ori32b; W.ori32b = f;
}

// ------------------------------------------------------------------ force kernel

// Minimum-image separation for the step kernel: k = rint(d * (1/L)) instead of
// rint(d / L).  The two differ only where d / L lies within a few ulp of a
// half-integer, that is at separations near L / 2, beyond every list radius (a
// periodic length exceeds twice the largest cutoff plus skin); every pair that can
// be in range gets the same k, hence the same separation bits, as the exact test.
__device__ __forceinline__ double minimg_fast(double d, double L, double iL) {
#pragma clang fp contract(off)
    const double k = __builtin_rint(d * iL);
    const double kl = k * L;
    return d - kl;
}

// Branch-free FP32 lipid-lipid law for the mixed-precision step kernel, on the
// separation (dx, dy, dz) = x_i - x_j with r2 = |d|^2 > 0.  Both radial branches are
// evaluated and selected (the repulsive core below r_min, the cos^(2 zeta) well above
// it); `on` masks the pair out (every coefficient and U zero) without a branch.
// With g = -t n_i - s n_j + sin(th0) (n_j - n_i) and k = dU/da / r, the force on i is
// -[(dU/dr - k g.e) e + k g], where g.e = -2 s t + sin(th0) (t - s), and the torque on i
// is n_i x g_i with g_i = -dU/da (n_j - (t + sin th0) e).  Both are returned as
// coefficients, so that the caller sums the terms along n_i, and forms the torque's
// cross product with n_i, once per particle instead of once per pair:
//   force on i  = -(A e + bi n_i + bj n_j),    g_i = cn n_j + ce e.
// Returns U; (ex, ey, ez) is the unit separation.
template <bool FAST>
__device__ __forceinline__ float lipid_coef(const DevParams &P, float dx, float dy, float dz, float r2, float nix,
                                            float niy, float niz, float njx, float njy, float njz, bool on,
                                            float &ex, float &ey, float &ez, float &A, float &bi, float &bj,
                                            float &cn, float &ce) {
    const float eps = (float)P.eps, mu = (float)P.mu, rmin = (float)P.r_min;
    const float st0 = FAST ? 0.0f : (float)P.st0;
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * rinv;
    ex = dx * rinv;
    ey = dy * rinv;
    ez = dz * rinv;
    const float s = nix * ex + niy * ey + niz * ez;
    const float t = njx * ex + njy * ey + njz * ez;
    const float c = nix * njx + niy * njy + niz * njz;
    float a = c - s * t;
    if (!FAST) a += st0 * (t - s) - st0 * st0;
    const float phi = mu * a + (1.0f - mu);
    // repulsive core, r < r_min: U = eps (q^2 - 2 q) + (1 - phi) eps with q = (r_min / r)^2
    const float q = (rmin * rmin) * (rinv * rinv);
    const float dUdrR = (4.0f * eps) * ((q - q * q) * rinv);
    const float dUdaR = -mu * eps;
    // attractive well, r_min <= r < r_c: x = (pi/2) u with u clamped to [0, 1]; the
    // hardware sine and cosine take revolutions, x / 2pi = u / 4
    const float w4 = 0.25f * (float)P.inv_w;
    const float arg = __builtin_amdgcn_fmed3f(r * w4 - rmin * w4, 0.0f, 0.25f);
    const float sx = __builtin_amdgcn_sinf(arg);
    const float cx = __builtin_amdgcn_cosf(arg);
    const float c2 = cx * cx;
    float cz1;                                           // cos^(2 zeta - 2)
    if (FAST) cz1 = (c2 * c2) * c2;
    else cz1 = ipow(c2, P.zeta - 1);
    const float c2z = cz1 * c2;                          // cos^(2 zeta)
    const float dUdrA = (phi * (float)P.dudr_k) * ((sx * cx) * cz1);
    const float dUdaA = (-mu * eps) * c2z;
    const bool rep = r < rmin;
    float dUdr = rep ? dUdrR : dUdrA;
    float dUda = rep ? dUdaR : dUdaA;
    float U = rep ? (eps * (q * q - 2.0f * q) + (1.0f - phi) * eps) : -eps * c2z * phi;
    dUdr = on ? dUdr : 0.0f;
    dUda = on ? dUda : 0.0f;
    U = on ? U : 0.0f;
    const float k = dUda * rinv;
    const float kt = k * t, ks = k * s;
    float ge2 = 2.0f * kt * s;                           // -k g.e
    if (!FAST) ge2 -= k * st0 * (t - s);
    A = dUdr + ge2;
    bi = -kt;                                            // k g = bi n_i + bj n_j
    bj = -ks;
    if (!FAST) {
        bi -= k * st0;
        bj += k * st0;
    }
    cn = -dUda;
    ce = dUda * (FAST ? t : t + st0);
    return U;
}

// LDS stage per 256-particle block (structure of arrays): FP64 positions, and either
// FP32 orientations with the type in w (mixed) or FP64 orientations and a type byte.
// The stage is the block's pruned partner set; entries beyond the LDS part (rare)
// are read from global memory.  Mixed mode keeps one more entry, a sentinel far
// from every particle with a padding type, which list padding points to (on periodic
// axes the wrap may bring it back into range, so periodic systems also test its type).
template <int MIXED>
struct Stage {
    static constexpr int lds = MIXED ? 640 : 800;
    static constexpr int ext = MIXED ? lds + 2 : lds;   // LDS entries (mixed: the sentinel and one pad)
    static constexpr int bytes = MIXED ? ext * (3 * 8 + 16) : lds * (6 * 8 + 1);
};
static_assert(Stage<1>::lds < SMAX && (Stage<1>::ext * 24) % 16 == 0, "mixed stage layout");
constexpr double SENTINEL = 1.0e8;    // sigma: the padding entry's coordinates (finite FP32 squares)
constexpr int PAD_TYPE = 3;           // the padding entry's type (a periodic wrap may bring it into range)

// One workgroup per 256 consecutive cell-sorted particles.  The block's pruned
// partners (its stage) are read once from HBM into LDS; lane i then walks column i of
// its chunk's pruned list of stage indices.
//  - Mixed mode: each row is evaluated without branches, two rows per trip.  The
//    FP64-formed separation is rounded to FP32 and its FP32 square decides the
//    neighbour test where it lies clear of the cutoff (beyond the FP32 rounding of the
//    square, a relative 4e-7 at most); in the band between, which a wavefront rarely
//    meets, the exact FP64 test of the neighbour-set definition decides.  The pair
//    law then runs in FP32.
//  - FP64 mode: every entry takes the exact FP64 test; the pair law runs in FP64.
// KICK: 0 stores F and tau; 1 also applies the closing half-kick of the step;
// 2 applies the closing half-kick and then, with the same force, the opening
// half-kick and drift of the next step (positions and orientations go to the
// second buffers, which the stats kernel then swaps in), without storing F, tau.
template <int MIXED, int ENERGY, int KICK, int FAST>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(MIXED ? 5 : 4))) void k_force(const SysDev *Sd, Maps L_maps, DevParams P, double dt) {
    using T = typename std::conditional<MIXED, float, double>::type;
    constexpr int SL = Stage<MIXED>::lds;
    constexpr int SX = Stage<MIXED>::ext;
    __shared__ __align__(16) unsigned char s_raw[Stage<MIXED>::bytes];
    double *s_x = reinterpret_cast<double *>(s_raw);
    double *s_y = s_x + SX;
    double *s_z = s_y + SX;
    F4 *s_n4 = reinterpret_cast<F4 *>(s_z + SX);                  // mixed
    double *s_nx = s_z + SL, *s_ny = s_nx + SL, *s_nz = s_ny + SL;        // FP64
    unsigned char *s_t = reinterpret_cast<unsigned char *>(s_nz + SL);    // FP64
    const int gb = xcd_group_block(blockIdx.x, gridDim.x);
    const int s = find_sys(L_maps.f, L_maps.nsys, gb);
    const SysDev &S = Sd[s];
    const int fb = gb - L_maps.f[s];
    // a split system's particle block runs as four blocks, one per chunk, whose four
    // waves take every fourth row of that chunk (block-uniform)
    const bool split = S.split != 0;
    const int lb = split ? fb >> 2 : fb;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int csub = split ? (fb & 3) : (tid >> 6);   // the chunk within the particle block
    const int chunk = lb * (BLOCK / WAVE) + csub;
    const int i = lb * BLOCK + csub * WAVE + lane;
    const bool valid = i < S.n;
    const int scnt = __builtin_amdgcn_readfirstlane(S.iscount[lb]);
    const int nlds = min(scnt, SL);                 // stage entries held in LDS
    // this lane's own particle, loaded while the stage is read
    const int traw = valid ? ldg(S.typ + i) : 0;
    const D4 pi = valid ? ld3(S.pos + i) : D4{0.0, 0.0, 0.0, 0.0};
    const D4 ni = valid ? ld3(S.ori + i) : D4{0.0, 0.0, 0.0, 0.0};
    // the stage: every thread's (at most three) slots first, then their records
    constexpr int SPT = (SL + BLOCK - 1) / BLOCK;
    for (int q0 = tid; q0 < nlds; q0 += SPT * BLOCK) {
        int slot[SPT];
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int q = q0 + k * BLOCK;
            slot[k] = q < nlds ? ldg(S.istage + (size_t)lb * SSTRIDE + q) : -1;
        }
#pragma unroll
        for (int k = 0; k < SPT; ++k) {
            const int q = q0 + k * BLOCK;
            if (slot[k] < 0) break;
            const V3 p = ldg(S.pos + slot[k]);
            s_x[q] = p.x;
            s_y[q] = p.y;
            s_z[q] = p.z;
            if constexpr (MIXED) {
                s_n4[q] = ldg(S.ori32 + slot[k]);       // w: the type's bits
            } else {
                const V3 o = S.ori[slot[k]];
                s_nx[q] = o.x;
                s_ny[q] = o.y;
                s_nz[q] = o.z;
                s_t[q] = ldg(S.typ + slot[k]) & TYP_MASK;
            }
        }
    }
    if (MIXED && tid == 0) {
        s_x[SL] = SENTINEL;
        s_y[SL] = SENTINEL;
        s_z[SL] = SENTINEL;
        s_n4[SL] = F4{0.0f, 0.0f, 1.0f, __int_as_float(PAD_TYPE)};
    }
    __syncthreads();
    if (chunk >= S.nchunk) return;
    const int ti = traw & TYP_MASK;
    const T nix = (T)ni.x, niy = (T)ni.y, niz = (T)ni.z;
    T fx = 0, fy = 0, fz = 0, tx = 0, ty = 0, tz = 0;
    double U = 0.0, W = 0.0;
    const int rows = __builtin_amdgcn_readfirstlane(min(S.ilk[chunk], MAXNB));   // wave-uniform
    // cutoff row of this particle's type, selected by the partner's type without
    // dynamic indexing; the periodic min-image only where the system has periodic axes
    const double rcA = ti == 0 ? P.rc2[0][0] : (ti == 1 ? P.rc2[1][0] : P.rc2[2][0]);
    const double rcB = ti == 0 ? P.rc2[0][1] : (ti == 1 ? P.rc2[1][1] : P.rc2[2][1]);
    const double rcC = ti == 0 ? P.rc2[0][2] : (ti == 1 ? P.rc2[1][2] : P.rc2[2][2]);
    const bool periodic = (S.per[0] | S.per[1] | S.per[2]) != 0;
    const double iLx = S.per[0] ? 1.0 / S.box[0] : 0.0, iLy = S.per[1] ? 1.0 / S.box[1] : 0.0,
                 iLz = S.per[2] ? 1.0 / S.box[2] : 0.0;

    // ---- mixed mode: branch-free rows, two per trip
    auto mixed_rows = [&](auto per_tag, auto part_tag, auto split_tag) {
        constexpr bool PER = decltype(per_tag)::value;
        constexpr bool PARTIAL = decltype(part_tag)::value;   // stage entries beyond the LDS part
        constexpr bool SPLIT = decltype(split_tag)::value;    // the four waves take every fourth pair of rows
        constexpr int UNR = 2;          // rows per trip (consecutive), evaluated side by side
        // The pruned lists are padded with 0xffff to an even row count in every lane, so
        // both rows of a trip are always valid entries or padding.
        const int nrow = (rows + 1) & ~1;
        const int r0 = SPLIT ? UNR * (tid >> 6) : 0;
        constexpr int tstride = SPLIT ? UNR * (BLOCK / WAVE) : UNR;
        const uint16_t *col = S.il16 + (size_t)chunk * MAXNB * CHUNK + r0 * CHUNK + lane;
        const int ntrip = nrow > r0 ? (nrow - r0 + tstride - 1) / tstride : 0;
        // this particle's row of the FP32 bounds, chosen by selects (no dynamic indexing
        // of the parameter block, which would go through scratch memory)
        auto row_of = [&](const float (&m)[3][3], int b) {
            return ti == 0 ? m[0][b] : (ti == 1 ? m[1][b] : m[2][b]);
        };
        const float loA = row_of(P.rc2lo, 0), loB = row_of(P.rc2lo, 1), loC = row_of(P.rc2lo, 2);
        const float hiA = row_of(P.rc2hi, 0), hiB = row_of(P.rc2hi, 1), hiC = row_of(P.rc2hi, 2);
        struct Rec {
            double x, y, z;
            float nx, ny, nz;
            int t;
        };
        auto fetch = [&](int e) {
            Rec c;
            if constexpr (PARTIAL) {
                if (e >= nlds && e < scnt) {            // stage entry beyond the LDS part
                    const int slot = ldg(S.istage + (size_t)lb * SSTRIDE + e);
                    const V3 p = ldg(S.pos + slot);
                    const F4 o = ldg(S.ori32 + slot);
                    c.x = p.x; c.y = p.y; c.z = p.z;
                    c.nx = o.x; c.ny = o.y; c.nz = o.z;
                    c.t = __float_as_int(o.w);
                    return c;
                }
            }
            // padding -> the sentinel (every entry below the LDS part when not PARTIAL)
            const int q = PARTIAL ? (e < nlds ? e : SL) : min(e, SL);
            c.x = s_x[q];
            c.y = s_y[q];
            c.z = s_z[q];
            const F4 nj = s_n4[q];
            c.nx = nj.x; c.ny = nj.y; c.nz = nj.z;
            c.t = __float_as_int(nj.w);
            return c;
        };
        // Software pipeline: the list entries of the next trip are loaded from global
        // memory while this trip's rows are evaluated (the lists carry padding rows past
        // the last chunk, so the load after the last trip stays in bounds).
        float sbi = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;   // sum of bi; of g_i - cn n_i
        int en[UNR];
        for (int q = 0; q < UNR; ++q) en[q] = ntrip > 0 ? (int)ldg(col + q * CHUNK) : 0xffff;
        for (int it = 0; it < ntrip; ++it) {
            Rec c[UNR];
            for (int q = 0; q < UNR; ++q) c[q] = fetch(en[q]);
            const uint16_t *nxt = col + (size_t)(it + 1) * tstride * CHUNK;
            for (int q = 0; q < UNR; ++q) en[q] = (int)ldg(nxt + q * CHUNK);
            // separations and the neighbour test of every row of the trip
            double dx[UNR], dy[UNR], dz[UNR];
            float fdx[UNR], fdy[UNR], fdz[UNR], r2[UNR];
            bool in[UNR], band[UNR], lip[UNR];
            bool anyband = false;
            for (int q = 0; q < UNR; ++q) {
                dx[q] = pi.x - c[q].x;
                dy[q] = pi.y - c[q].y;
                dz[q] = pi.z - c[q].z;
                if constexpr (PER) {
                    if (S.per[0]) dx[q] = minimg_fast(dx[q], S.box[0], iLx);
                    if (S.per[1]) dy[q] = minimg_fast(dy[q], S.box[1], iLy);
                    if (S.per[2]) dz[q] = minimg_fast(dz[q], S.box[2], iLz);
                }
                fdx[q] = (float)dx[q];
                fdy[q] = (float)dy[q];
                fdz[q] = (float)dz[q];
                r2[q] = fdx[q] * fdx[q] + fdy[q] * fdy[q] + fdz[q] * fdz[q];
                const int tj = c[q].t;
                const float lo = FAST ? (tj == 0 ? loA : loB) : sel_cutf(tj, loA, loB, loC);
                const float hi = FAST ? (tj == 0 ? hiA : hiB) : sel_cutf(tj, hiA, hiB, hiC);
                in[q] = r2[q] < lo;
                band[q] = !in[q] && r2[q] < hi;
                if constexpr (PER) {            // the wrapped sentinel may land anywhere
                    in[q] = in[q] && tj != PAD_TYPE;
                    band[q] = band[q] && tj != PAD_TYPE;
                }
                anyband = anyband || band[q];
                lip[q] = (ti | tj) == 0;
            }
            if (__builtin_expect(__ballot(anyband) != 0ull, 0)) {
#pragma clang fp contract(off)
                // FP32 rounding cannot decide: the exact test of the neighbour-set definition
                for (int q = 0; q < UNR; ++q) {
                    const double d2 = (dx[q] * dx[q] + dy[q] * dy[q]) + dz[q] * dz[q];
                    if (band[q]) in[q] = d2 < sel_cut(c[q].t, rcA, rcB, rcC);
                }
            }
            // the pair law of every row, in one block of straight-line code, as coefficients
            float ex[UNR], ey[UNR], ez[UNR], A[UNR], bi[UNR], bj[UNR], cn[UNR], ce[UNR], u[UNR];
            bool anywca = false;
            for (int q = 0; q < UNR; ++q) {
                in[q] = in[q] && valid;
                u[q] = lipid_coef<FAST>(P, fdx[q], fdy[q], fdz[q], r2[q], nix, niy, niz, c[q].nx, c[q].ny, c[q].nz,
                                        in[q] && lip[q], ex[q], ey[q], ez[q], A[q], bi[q], bj[q], cn[q], ce[q]);
                anywca = anywca || (in[q] && !lip[q]);
            }
            for (int q = 0; q < UNR; ++q) {
                fx = fmaf(-A[q], ex[q], fx);
                fy = fmaf(-A[q], ey[q], fy);
                fz = fmaf(-A[q], ez[q], fz);
                fx = fmaf(-bj[q], c[q].nx, fx);
                fy = fmaf(-bj[q], c[q].ny, fy);
                fz = fmaf(-bj[q], c[q].nz, fz);
                sbi += bi[q];
                // the torque n_i x g_i with g_i = cn n_j + ce e: n_i x n_i = 0, so the sum
                // takes cn (n_j - n_i) + ce e instead, without g_i's large part along n_i
                // (which the FP32 sum would round before the cross product cancels it)
                gx = fmaf(cn[q], c[q].nx - nix, gx);
                gy = fmaf(cn[q], c[q].ny - niy, gy);
                gz = fmaf(cn[q], c[q].nz - niz, gz);
                gx = fmaf(ce[q], ex[q], gx);
                gy = fmaf(ce[q], ey[q], gy);
                gz = fmaf(ce[q], ez[q], gz);
                if (ENERGY) {
                    const float ax = A[q] * ex[q] + bi[q] * nix + bj[q] * c[q].nx;
                    const float ay = A[q] * ey[q] + bi[q] * niy + bj[q] * c[q].ny;
                    const float az = A[q] * ez[q] + bi[q] * niz + bj[q] * c[q].nz;
                    U += 0.5 * (double)u[q];
                    W -= 0.5 * (dx[q] * (double)ax + dy[q] * (double)ay + dz[q] * (double)az);
                }
            }
            if (__builtin_expect(__ballot(anywca) != 0ull, 0)) {
                for (int q = 0; q < UNR; ++q) {
                    const bool wca = in[q] && !lip[q];
                    float bx = 0.0f, by = 0.0f, bz = 0.0f;
                    const float uw = wca_pair<float>(P, wca ? fdx[q] : 2.0f, fdy[q], fdz[q], bx, by, bz);
                    if (wca) {
                        fx += bx;
                        fy += by;
                        fz += bz;
                        if (ENERGY) {
                            U += 0.5 * (double)uw;
                            W += 0.5 * (dx[q] * (double)bx + dy[q] * (double)by + dz[q] * (double)bz);
                        }
                    }
                }
            }
        }
        // the terms along n_i, and the torque n_i x (sum of the g_i - cn n_i)
        fx -= sbi * nix;
        fy -= sbi * niy;
        fz -= sbi * niz;
        tx += niy * gz - niz * gy;
        ty += niz * gx - nix * gz;
        tz += nix * gy - niy * gx;
    };

    // ---- FP64 mode: exact test on every entry, FP64 pair law
    auto fp64_rows = [&](auto per_tag, auto part_tag, auto split_tag) {
        constexpr bool PER = decltype(per_tag)::value;
        constexpr bool PARTIAL = decltype(part_tag)::value;
        constexpr bool SPLIT = decltype(split_tag)::value;
        constexpr int rstep = SPLIT ? BLOCK / WAVE : 1;
        const int r0 = SPLIT ? (tid >> 6) : 0;
        // Software pipeline: the list entry of row r+4 is fetched from global memory and
        // the stage record of row r+1 from LDS while row r is evaluated.
        const uint16_t *col = S.il16 + (size_t)chunk * MAXNB * CHUNK + r0 * CHUNK + lane;
        const int cstep = rstep * CHUNK;
        const int nr = rows > r0 ? (rows - r0 + rstep - 1) / rstep : 0;
        int e_cur = (valid && nr > 0) ? (int)ldg(col) : 0xffff;
        int e_nxt = (valid && nr > 1) ? (int)ldg(col + cstep) : 0xffff;
        int e_n2 = (valid && nr > 2) ? (int)ldg(col + 2 * cstep) : 0xffff;
        int e_n3 = (valid && nr > 3) ? (int)ldg(col + 3 * cstep) : 0xffff;
        struct Rec {
            double x, y, z;
            T nx, ny, nz;
            int t;
        };
        auto fetch = [&](int e) {
            Rec c;
            if constexpr (PARTIAL) {
                if (e >= nlds && e < scnt) {
                    const int slot = ldg(S.istage + (size_t)lb * SSTRIDE + e);
                    const V3 p = ldg(S.pos + slot);
                    const V3 o = ldg(S.ori + slot);
                    c.x = p.x; c.y = p.y; c.z = p.z;
                    c.nx = o.x; c.ny = o.y; c.nz = o.z;
                    c.t = ldg(S.typ + slot) & TYP_MASK;
                    return c;
                }
            }
            const int q = e < nlds ? e : 0;             // in-bounds dummy for padding entries
            c.x = s_x[q];
            c.y = s_y[q];
            c.z = s_z[q];
            c.nx = s_nx[q]; c.ny = s_ny[q]; c.nz = s_nz[q];
            c.t = s_t[q];
            return c;
        };
        Rec rec = fetch(e_cur);
        for (int r = 0; r < nr; ++r) {
            const int e = e_cur;
            const Rec c = rec;
            e_cur = e_nxt;
            e_nxt = e_n2;
            e_n2 = e_n3;
            e_n3 = (valid && r + 4 < nr) ? (int)ldg(col + (r + 4) * cstep) : 0xffff;
            rec = fetch(e_cur);
            if (e >= scnt) continue;
            const int tj = c.t;
            double dx, dy, dz, d2;
            if constexpr (PER) {
                d2 = dist2_exact(S, pi.x, pi.y, pi.z, c.x, c.y, c.z, dx, dy, dz);
            } else {
                d2 = dist2_open(pi.x, pi.y, pi.z, c.x, c.y, c.z, dx, dy, dz);
            }
            const double rc2 = sel_cut(tj, rcA, rcB, rcC);
            if (!(d2 < rc2)) continue;
            T ax = 0, ay = 0, az = 0, u;
            if ((ti | tj) == 0)
                u = lipid_pair<T, FAST>(P, (T)dx, (T)dy, (T)dz, nix, niy, niz, c.nx, c.ny, c.nz, ax, ay, az, tx, ty,
                                        tz);
            else
                u = wca_pair<T>(P, (T)dx, (T)dy, (T)dz, ax, ay, az);
            fx += ax;
            fy += ay;
            fz += az;
            if (ENERGY) {
                U += 0.5 * (double)u;
                W += 0.5 * (dx * (double)ax + dy * (double)ay + dz * (double)az);
            }
        }
    };

    if (scnt >= 0) {
        // block-uniform choices: periodic min-image, whether the stage overflows the LDS
        // part, and the row split, so ordinary blocks carry no per-entry test
        auto dispatch = [&](auto per_tag, auto part_tag) {
            if constexpr (MIXED) {
                if (split) mixed_rows(per_tag, part_tag, std::true_type{});
                else mixed_rows(per_tag, part_tag, std::false_type{});
            } else {
                if (split) fp64_rows(per_tag, part_tag, std::true_type{});
                else fp64_rows(per_tag, part_tag, std::false_type{});
            }
        };
        if (scnt > SL) {
            if (periodic) dispatch(std::true_type{}, std::true_type{});
            else dispatch(std::false_type{}, std::true_type{});
        } else {
            if (periodic) dispatch(std::true_type{}, std::false_type{});
            else dispatch(std::false_type{}, std::false_type{});
        }
    } else {
        // block whose partners did not fit a stage: its (unpruned) lists hold global slots
        const int32_t *col = S.nl + (size_t)chunk * MAXNB * CHUNK + lane;
        const int r0 = split ? (tid >> 6) : 0, rstep = split ? BLOCK / WAVE : 1;
        for (int r = r0; r < rows; r += rstep) {
            const int j = valid ? col[r * CHUNK] : -1;
            if (j < 0 || j >= S.n) continue;
            const D4 pj = ldpos(S, j);
            const int tj = (int)pj.w;
            double dx, dy, dz;
            const double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
            if (!(d2 < P.rc2[ti][tj])) continue;
            T ax = 0, ay = 0, az = 0;
            T u;
            if ((ti | tj) == 0) {
                const V3 nj = S.ori[j];
                u = lipid_pair<T, FAST>(P, (T)dx, (T)dy, (T)dz, nix, niy, niz, (T)nj.x, (T)nj.y, (T)nj.z, ax, ay, az,
                                        tx, ty, tz);
            } else {
                u = wca_pair<T>(P, (T)dx, (T)dy, (T)dz, ax, ay, az);
            }
            fx += ax;
            fy += ay;
            fz += az;
            if (ENERGY) {
                U += 0.5 * (double)u;
                W += 0.5 * (dx * (double)ax + dy * (double)ay + dz * (double)az);
            }
        }
    }
    if (split) {
        // the four waves' partial sums, added in wave order by wave 0, which goes on
        // with the chunk's particles; the stage is free again
        __syncthreads();
        T *red = reinterpret_cast<T *>(s_raw);
        double *redd = reinterpret_cast<double *>(s_raw + 6 * BLOCK * sizeof(T));
        const int wv = tid >> 6;
        const T mine[6] = {fx, fy, fz, tx, ty, tz};
        for (int q = 0; q < 6; ++q) red[q * BLOCK + wv * WAVE + lane] = mine[q];
        if (ENERGY) {
            redd[wv * WAVE + lane] = U;
            redd[BLOCK + wv * WAVE + lane] = W;
        }
        __syncthreads();
        if (wv != 0) return;
        T sum[6];
        for (int q = 0; q < 6; ++q)
            sum[q] = ((red[q * BLOCK + lane] + red[q * BLOCK + WAVE + lane]) + red[q * BLOCK + 2 * WAVE + lane]) +
                     red[q * BLOCK + 3 * WAVE + lane];
        fx = sum[0]; fy = sum[1]; fz = sum[2];
        tx = sum[3]; ty = sum[4]; tz = sum[5];
        if (ENERGY) {
            U = ((redd[lane] + redd[WAVE + lane]) + redd[2 * WAVE + lane]) + redd[3 * WAVE + lane];
            W = ((redd[BLOCK + lane] + redd[BLOCK + WAVE + lane]) + redd[BLOCK + 2 * WAVE + lane]) +
                redd[BLOCK + 3 * WAVE + lane];
        }
    }
    double Fx = (double)fx, Fy = (double)fy, Fz = (double)fz;
    D4 v = {0.0, 0.0, 0.0, 0.0}, w = {0.0, 0.0, 0.0, 0.0};
    double disp2 = 0.0, disp2p = 0.0, vmax2 = 0.0;
    bool bad = false;
    D4 Tq = {(double)tx, (double)ty, (double)tz, 0.0};
    double vsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        // the own-state loads first, so that they are in flight during the bond lookups
        if (KICK || ENERGY) {
            v = ld3(S.vel + i);
            if (ti == 0) w = ld3(S.angv + i);        // zero for protein beads
        }
        const F3 xb = KICK == 2 ? ldg(S.xb + i) : F3{0.f, 0.f, 0.f};
        const F3 xp = KICK == 2 ? ldg(S.xp + i) : F3{0.f, 0.f, 0.f};
        // bonds of this particle (CSR by caller id), FP64 in both modes; the table is
        // looked up only for particles flagged as bonded
        const bool bonded = (traw & TYP_BONDED) != 0;
        const int g = (bonded || P.thermo_on) ? S.gid[i] : 0;
        const int qb = bonded ? S.bstart[g] : 0, qe = bonded ? S.bstart[g + 1] : 0;
        for (int q = qb; q < qe; ++q) {
            const int j = S.slot[S.bpart[q]];
            const D4 pj = ld3(S.pos + j);
            double dx, dy, dz;
            const double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
            const double r = sqrt(d2);
            const double ext = r - S.br0[q];
            const double f = (r > 0.0) ? -P.k_bond * ext / r : 0.0;
            Fx += f * dx;
            Fy += f * dy;
            Fz += f * dz;
            if (ENERGY) {
                U += 0.25 * P.k_bond * ext * ext;
                W += 0.5 * f * d2;
            }
        }
        if (P.vol_on && ti == 0) volume_term(S.sc, pi, ni, Fx, Fy, Fz, Tq);
        if (KICK != 2) {
            S.frc[i] = V3{Fx, Fy, Fz};
            st3(S.trq + i, Tq);
        }
        if (KICK) {
            const double h = 0.5 * dt * P.inv_mass[ti];
            const double hw = 0.5 * dt * P.inv_inertia;
            half_kick(v, h, Fx, Fy, Fz);
            if (ti == 0) half_kick(w, hw, Tq.x, Tq.y, Tq.z);
            if (P.thermo_on) langevin_update(P, g, S.sc->step, ti, ni, v, w);
            if (P.quench_on) {
                project_along(v, Fx, Fy, Fz);
                if (ti == 0) project_along(w, Tq.x, Tq.y, Tq.z);
            }
            if (KICK == 1) {
                st3(S.vel + i, v);
                if (ti == 0) st3(S.angv + i, w);
            } else {
                D4 vn = v, wn = w, xn = pi;
                half_kick(vn, h, Fx, Fy, Fz);
                if (P.quench_on) cap_move(vn, dt, P.quench_max);
                drift_pos(xn, vn, dt);
                st3(S.vel + i, vn);
                st3(S.pos2 + i, xn);
                D4 on = ni;
                if (ti == 0) {
                    half_kick(wn, hw, Tq.x, Tq.y, Tq.z);
                    if (P.quench_on) cap_move(wn, dt, P.quench_max);
                    st3(S.angv + i, wn);
                    on = rotor_drift(ni, wn, dt);
                }
                st3(S.ori2 + i, on);
                S.ori32b[i] = F4{(float)on.x, (float)on.y, (float)on.z, __int_as_float(ti)};
                drift_measures(xn, vn, xb, xp, disp2, disp2p, vmax2, bad);
                if (P.vol_on && ti == 0) volume_terms(xn, on, vsum);
            }
        }
    }
    if (KICK == 2) {
        drift_stats(S, lb, csub, disp2, vmax2, disp2p, bad);
        if (P.vol_on) volume_chunk_store(S, chunk, vsum);
        if (split) publish_split(const_cast<SysDev &>(S), S.nchunk, disp2, vmax2, disp2p);   // a workgroup per chunk
    }
    if (ENERGY) {
        // per-chunk partials of U, W, KE, sum F and sum (r x F + tau), reduced across
        // the wavefront in a fixed butterfly (deterministic)
        double vals[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (valid) {
            const double m = 1.0 / P.inv_mass[ti];
            double ke = 0.5 * m * (v.x * v.x + v.y * v.y + v.z * v.z);
            if (ti == 0) ke += 0.5 / P.inv_inertia * (w.x * w.x + w.y * w.y + w.z * w.z);
            vals[0] = U;
            vals[1] = W;
            vals[2] = ke;
            vals[3] = Fx;
            vals[4] = Fy;
            vals[5] = Fz;
            vals[6] = pi.y * Fz - pi.z * Fy + Tq.x;
            vals[7] = pi.z * Fx - pi.x * Fz + Tq.y;
            vals[8] = pi.x * Fy - pi.y * Fx + Tq.z;
        }
        for (int q = 0; q < 9; ++q) vals[q] = wave_sum(vals[q]);
        if (lane == 0)
            for (int q = 0; q < 9; ++q) S.epart[chunk * 9 + q] = vals[q];
    }
}

template <int MIXED, int ENERGY, int KICK>
static void launch_force_t(const LaunchCtx &L, double dt) {
    // FAST: the default pair-law constants, and one cutoff for both protein types
    bool fast = L.prm.zeta == 4 && L.prm.st0 == 0.0;
    for (int t = 0; t < 3; ++t) fast = fast && L.prm.rc2[t][1] == L.prm.rc2[t][2];
    if (fast)
        hipLaunchKernelGGL((k_force<MIXED, ENERGY, KICK, 1>), dim3(L.nblk_f), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm,
                           dt);
    else
        hipLaunchKernelGGL((k_force<MIXED, ENERGY, KICK, 0>), dim3(L.nblk_f), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm,
                           dt);
}

void launch_force(const LaunchCtx &L, int mixed, int energy, int kick, double dt) {
    if (L.prm.vol_on) launch_volume_reduce(L);   // V of the current state from its lipid sums
    if (kick == 2) {
        if (mixed) launch_force_t<1, 0, 2>(L, dt);
        else launch_force_t<0, 0, 2>(L, dt);
        return;
    }
    const int key = (mixed ? 4 : 0) | (energy ? 2 : 0) | (kick ? 1 : 0);
    switch (key) {
        case 0: launch_force_t<0, 0, 0>(L, dt); break;
        case 1: launch_force_t<0, 0, 1>(L, dt); break;
        case 2: launch_force_t<0, 1, 0>(L, dt); break;
        case 3: launch_force_t<0, 1, 1>(L, dt); break;
        case 4: launch_force_t<1, 0, 0>(L, dt); break;
        case 5: launch_force_t<1, 0, 1>(L, dt); break;
        case 6: launch_force_t<1, 1, 0>(L, dt); break;
        default: launch_force_t<1, 1, 1>(L, dt); break;
    }
}

// ------------------------------------------------------------------ kick + drift

// v += dt/2m F, omega += dt/2I tau (lipids); x += dt v; n rotated about omega by
// |omega| dt (Rodrigues) and renormalised.  Tracks the largest displacement since
// the last cell build and the largest drift speed, per system.
__global__ __launch_bounds__(BLOCK) void k_kick_drift(const SysDev *Sd, Maps L_maps, DevParams P, double dt) {
    const int s = find_sys(L_maps.p, L_maps.nsys, blockIdx.x);
    const SysDev &S = Sd[s];
    const int lb = blockIdx.x - L_maps.p[s];
    const int i = lb * BLOCK + threadIdx.x;
    double disp2 = 0.0, disp2p = 0.0, v2 = 0.0;
    bool bad = false;
    double vsum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < S.n) {
        D4 p = ldpos(S, i), v = ld3(S.vel + i);
        const D4 f = ld3(S.frc + i);
        const int t = (int)p.w;
        const double h = 0.5 * dt * P.inv_mass[t];
        half_kick(v, h, f.x, f.y, f.z);
        if (P.quench_on) cap_move(v, dt, P.quench_max);
        drift_pos(p, v, dt);
        st3(S.vel + i, v);
        st3(S.pos + i, p);
        if (t == 0) {
            D4 w = ld3(S.angv + i);
            const D4 tq = ld3(S.trq + i);
            const double hw = 0.5 * dt * P.inv_inertia;
            half_kick(w, hw, tq.x, tq.y, tq.z);
            if (P.quench_on) cap_move(w, dt, P.quench_max);
            const D4 n = rotor_drift(ld3(S.ori + i), w, dt);
            st3(S.angv + i, w);
            st3(S.ori + i, n);
            S.ori32[i] = F4{(float)n.x, (float)n.y, (float)n.z, __int_as_float(t)};
            if (P.vol_on) volume_terms(p, n, vsum);
        }
        drift_measures(p, v, S.xb[i], S.xp[i], disp2, disp2p, v2, bad);
    }
    drift_stats(S, lb, (threadIdx.x >> 6) & 3, disp2, v2, disp2p, bad);
    if (P.vol_on && i / CHUNK < S.nchunk) volume_chunk_store(S, i / CHUNK, vsum);
}

// Largest displacements since the last build and since the last prune, and the
// largest drift speed, per system, from the per-wavefront partials of a drift, three
// per 64-particle chunk.  STATS_BLOCKS blocks per system fold their share with an
// unsigned atomic max on the bits (non-negative doubles order like their bit
// patterns); the last one publishes the result.  swap: after the drift fused into
// the force kernel, which wrote the second position / orientation buffers; the last
// block swaps them in.
constexpr int STATS_BLOCKS = 64;

__global__ __launch_bounds__(256) void k_stats_reduce(SysDev *Sd, int nsys, int swap) {
    SysDev &S = Sd[blockIdx.x / STATS_BLOCKS];
    if (swap && S.split) return;          // the step kernel published this small system's drift
    const int part = blockIdx.x % STATS_BLOCKS;
    const int per = (S.nchunk + STATS_BLOCKS - 1) / STATS_BLOCKS;
    const int c0 = part * per, c1 = min(S.nchunk, c0 + per);
    double d = 0.0, v = 0.0, dp = 0.0;
    for (int c = c0 + (int)threadIdx.x; c < c1; c += blockDim.x) {
        d = fmax(d, S.bred[3 * c]);
        v = fmax(v, S.bred[3 * c + 1]);
        dp = fmax(dp, S.bred[3 * c + 2]);
    }
    d = wave_maxd(d);
    v = wave_maxd(v);
    dp = wave_maxd(dp);
    __shared__ double s_m[3][4];
    if ((threadIdx.x & 63) == 0) {
        s_m[0][threadIdx.x >> 6] = d;
        s_m[1][threadIdx.x >> 6] = v;
        s_m[2][threadIdx.x >> 6] = dp;
    }
    __syncthreads();
    if (threadIdx.x == 0 && S.n > 0) {
        d = fmax(fmax(s_m[0][0], s_m[0][1]), fmax(s_m[0][2], s_m[0][3]));
        v = fmax(fmax(s_m[1][0], s_m[1][1]), fmax(s_m[1][2], s_m[1][3]));
        dp = fmax(fmax(s_m[2][0], s_m[2][1]), fmax(s_m[2][2], s_m[2][3]));
        SysScal *sc = S.sc;
        if (c1 > c0) {
            atomicMax(&sc->maxdisp2, dbits(d));
            atomicMax(&sc->maxv2, dbits(v));
            atomicMax(&sc->maxdisp2p, dbits(dp));
        }
        __threadfence();
        if (atomicAdd(&sc->parts_done, 1u) == STATS_BLOCKS - 1) {
            __threadfence();
            publish_drift(sc, S.hstat);
            sc->parts_done = 0;
            if (swap) swap_drift(S);
        }
    }
}

void launch_kick_drift(const LaunchCtx &L, double dt) {
    hipLaunchKernelGGL(k_kick_drift, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm, dt);
    hipLaunchKernelGGL(k_stats_reduce, dim3(L.nsys * STATS_BLOCKS), dim3(256), 0, L.st, L.Sw, L.nsys, 0);
}

void launch_drift_stats_swap(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_stats_reduce, dim3(L.nsys * STATS_BLOCKS), dim3(256), 0, L.st, L.Sw, L.nsys, 1);
}

// ------------------------------------------------------------------ energy reduction

// Fixed-order sum of the per-chunk partials of each system (one block per system).
__global__ __launch_bounds__(256) void k_reduce_energy(const SysDev *Sd, int nsys, int vol_on) {
    const SysDev &S = Sd[blockIdx.x];
    __shared__ double sh[9][4];
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = threadIdx.x; c < S.nchunk; c += blockDim.x)
        for (int q = 0; q < 9; ++q) acc[q] += S.epart[c * 9 + q];
    for (int q = 0; q < 9; ++q) acc[q] = wave_sum(acc[q]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 9; ++q) sh[q][w] = acc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 9; ++q) S.sc->energy[q] = ((sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]));
        if (vol_on) S.sc->energy[0] += S.sc->volU;
    }
}

void launch_reduce_energy(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_reduce_energy, dim3(L.nsys), dim3(256), 0, L.st, L.S, L.nsys, L.prm.vol_on);
}

// ------------------------------------------------------------------ volume

// The lipid sums per chunk of the current state, for force evaluations that no
// drift precedes (a freshly loaded system).
__global__ __launch_bounds__(BLOCK) void k_volume_partials(const SysDev *Sd, Maps L_maps) {
    const int s = find_sys(L_maps.p, L_maps.nsys, blockIdx.x);
    const SysDev &S = Sd[s];
    const int lb = blockIdx.x - L_maps.p[s];
    const int i = lb * BLOCK + threadIdx.x;
    if (i / CHUNK >= S.nchunk) return;           // whole wavefronts past the last chunk
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i < S.n) {
        const D4 p = ldpos(S, i);
        if (p.w == 0.0) volume_terms(p, ld3(S.ori + i), v);
    }
    volume_chunk_store(S, i / CHUNK, v);
}

// Two fixed-order levels: VR1 blocks per system each sum a contiguous range of
// chunk totals into vred[b * 8 + q]; one block per system then sums those and
// derives V = a_L/3 (sum x.n - (sum x).(sum n) / N_L), U_V = k_V/2 (V - V0)^2 / V0
// and the force constant dU_V/dV a_L/3.  V0 is the given target, else the first V.
constexpr int VR1 = 32;

__global__ __launch_bounds__(256) void k_volume_reduce1(const SysDev *Sd, int nsys) {
    const SysDev &S = Sd[blockIdx.x / VR1];
    const int part = blockIdx.x % VR1;
    const int per = (S.nchunk + VR1 - 1) / VR1;
    const int c0 = part * per, c1 = min(S.nchunk, c0 + per);
    __shared__ double sh[8][4];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = c0 + (int)threadIdx.x; c < c1; c += 256)
        for (int q = 0; q < 8; ++q) acc[q] += S.vpart[(size_t)q * S.nchunk + c];
    for (int q = 0; q < 8; ++q) acc[q] = wave_sum(acc[q]);
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0)
        for (int q = 0; q < 8; ++q) sh[q][w] = acc[q];
    __syncthreads();
    if (threadIdx.x < 8 && S.n > 0) {
        const int q = threadIdx.x;
        S.vred[part * 8 + q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
    }
}

__global__ __launch_bounds__(64) void k_volume_reduce2(const SysDev *Sd, int nsys, DevParams P) {
    const SysDev &S = Sd[blockIdx.x];
    if (threadIdx.x != 0 || S.n == 0) return;
    double t[8];
    for (int q = 0; q < 8; ++q) {
        double a = 0.0;
        for (int b = 0; b < VR1; ++b) a += S.vred[b * 8 + q];
        t[q] = a;
    }
    SysScal *sc = S.sc;
    const double cnt = t[7];
    if (cnt == 0.0) {
        sc->volV = 0.0; sc->volkap = 0.0; sc->volU = 0.0;
        for (int a = 0; a < 3; ++a) { sc->xbar[a] = 0.0; sc->nbar[a] = 0.0; }
        return;
    }
    const double V = P.vol_a3 * (t[0] - (t[1] * t[4] + t[2] * t[5] + t[3] * t[6]) / cnt);
    sc->volV = V;
    for (int a = 0; a < 3; ++a) { sc->xbar[a] = t[1 + a] / cnt; sc->nbar[a] = t[4 + a] / cnt; }
    if (sc->vol0 == 0.0) sc->vol0 = P.vol_target > 0.0 ? P.vol_target : V;
    const double V0 = sc->vol0;
    if (P.vol_on && V0 > 0.0) {
        sc->volkap = P.vol_k * (V - V0) / V0 * P.vol_a3;
        sc->volU = 0.5 * P.vol_k * (V - V0) * (V - V0) / V0;
    } else {
        sc->volkap = 0.0;
        sc->volU = 0.0;
    }
}

void launch_volume_partials(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_volume_partials, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps);
}

void launch_volume_reduce(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_volume_reduce1, dim3(L.nsys * VR1), dim3(256), 0, L.st, L.S, L.nsys);
    hipLaunchKernelGGL(k_volume_reduce2, dim3(L.nsys), dim3(64), 0, L.st, L.S, L.nsys, L.prm);
}

// ------------------------------------------------------------------ outputs in caller order

__global__ void k_scatter_state(const SysDev *Sd, int s, double *x, double *n, double *v, double *w) {
    const SysDev &S = Sd[s];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    const int g = S.gid[i];
    if (x) { V3 p = S.pos[i]; x[3 * g] = p.x; x[3 * g + 1] = p.y; x[3 * g + 2] = p.z; }
    if (n) { V3 p = S.ori[i]; n[3 * g] = p.x; n[3 * g + 1] = p.y; n[3 * g + 2] = p.z; }
    if (v) { V3 p = S.vel[i]; v[3 * g] = p.x; v[3 * g + 1] = p.y; v[3 * g + 2] = p.z; }
    if (w) { V3 p = S.angv[i]; w[3 * g] = p.x; w[3 * g + 1] = p.y; w[3 * g + 2] = p.z; }
}

void launch_scatter_state(const LaunchCtx &L, int sys, double *x, double *n, double *v, double *w, int count) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_scatter_state, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, L.st, L.S, sys, x, n, v, w);
}

__global__ void k_scatter_forces(const SysDev *Sd, int s, double *F, double *T) {
    const SysDev &S = Sd[s];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    const int g = S.gid[i];
    if (F) { V3 p = S.frc[i]; F[3 * g] = p.x; F[3 * g + 1] = p.y; F[3 * g + 2] = p.z; }
    if (T) { V3 p = S.trq[i]; T[3 * g] = p.x; T[3 * g + 1] = p.y; T[3 * g + 2] = p.z; }
}

void launch_scatter_forces(const LaunchCtx &L, int sys, double *F, double *T, int count) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_scatter_forces, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, L.st, L.S, sys, F, T);
}

// ------------------------------------------------------------------ neighbour-set export

// Pairs (gid_i < gid_j) of the pruned lists the step kernel walks that pass the
// exact FP64 test, appended in any order (one atomic per wavefront).
// Pruned blocks keep indices into their pruned stage in the 16-bit lists (0xffff
// pads); the others keep global slots in the 32-bit lists (-1 pads).
__device__ __forceinline__ int entry_slot(const SysDev &S, int blk, int scnt, int chunk, int lane, int r) {
    const size_t at = (size_t)chunk * MAXNB * CHUNK + (size_t)r * CHUNK + lane;
    if (scnt >= 0) {
        const int e = S.il16[at];
        return e < scnt ? S.istage[(size_t)blk * SSTRIDE + e] : -1;
    }
    return S.nl[at];
}

__global__ void k_export_pairs(const SysDev *Sd, int s, DevParams P, int32_t *out, int64_t cap, int32_t *count) {
    const SysDev &S = Sd[s];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < S.n;
    const int chunk = i / CHUNK, lane = i % CHUNK, blk = i / BLOCK;
    D4 pi = {0, 0, 0, 0};
    int ti = 0, gi = 0, rows = 0, scnt = -1;
    if (valid) {
        pi = ldpos(S, i);
        ti = (int)pi.w;
        gi = S.gid[i];
        rows = min(S.ilk[chunk], MAXNB);
        scnt = S.iscount[blk];
    }
    int mine = 0;
    for (int pass = 0; pass < 2; ++pass) {
        int base = 0;
        if (pass == 1) {
            int tot = mine, ex = mine;
            for (int o = 1; o < 64; o <<= 1) {
                int y = __shfl_up(ex, o);
                if (lane_id_f() >= o) ex += y;
            }
            tot = __shfl(ex, 63);
            ex -= mine;
            int wb = 0;
            if (lane_id_f() == 0 && tot > 0) wb = atomicAdd(count, tot);
            base = __shfl(wb, 0) + ex;
        }
        int k = 0;
        for (int r = 0; r < rows; ++r) {
            const int j = entry_slot(S, blk, scnt, chunk, lane, r);
            if (j < 0 || j >= S.n) continue;
            const int gj = S.gid[j];
            if (gj <= gi) continue;
            const D4 pj = ldpos(S, j);
            double dx, dy, dz;
            const double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
            if (d2 < P.rc2[ti][(int)pj.w]) {
                if (pass == 1 && (int64_t)(base + k) < cap) {
                    out[2 * (base + k)] = gi;
                    out[2 * (base + k) + 1] = gj;
                }
                ++k;
            }
        }
        mine = k;
    }
}

void launch_export_pairs(const LaunchCtx &L, int sys, int count, int32_t *out, int64_t cap, int32_t *counter) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_export_pairs, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, L.st, L.S, sys, L.prm, out,
                       cap, counter);
}

// ------------------------------------------------------------------ allocation-free pair export

// Staging for the pair export of rbc_get_pairs_noalloc, for callers that cannot
// allocate device memory: a counter in the first word, then up to PAIR_SCRATCH_PAIRS
// pairs from byte 256 on.  Each device holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns on that
// device (pair_scratch_address), never through the array's name.
constexpr int64_t PAIR_SCRATCH_BYTES = 32ll << 20;
static __device__ __align__(256) int32_t scratch[PAIR_SCRATCH_BYTES / 4];

__global__ void k_zero_counter(int32_t *p) {
    if (threadIdx.x == 0) *p = 0;
}

hipError_t pair_scratch_address(int device, void **out) {
    static std::mutex mtx;
    static void *addr[64] = {};
    if (device < 0 || device >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mtx);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;      // the caller makes the device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

void launch_zero_counter(const LaunchCtx &L, int32_t *p) {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, L.st, p);
}

}  // namespace rbc
