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

// ------------------------------------------------------------------ pair laws

// Lipid-lipid orientation-dependent law; d = x_i - x_j.  Adds the force and torque
// on i and returns U (with dU/dr, dU/da and the gradient projection written out).
template <class T>
__device__ __forceinline__ T lipid_pair(const DevParams &P, T dx, T dy, T dz, T nix, T niy, T niz, T njx, T njy,
                                        T njz, T &fx, T &fy, T &fz, T &tx, T &ty, T &tz);

template <>
__device__ __forceinline__ float lipid_pair<float>(const DevParams &P, float dx, float dy, float dz, float nix,
                                                   float niy, float niz, float njx, float njy, float njz, float &fx,
                                                   float &fy, float &fz, float &tx, float &ty, float &tz) {
    const float eps = (float)P.eps, mu = (float)P.mu, st0 = (float)P.st0, rmin = (float)P.r_min;
    const float rc = (float)P.rc_lipid;
    const float inv_w = 1.0f / (rc - rmin);
    float r2 = dx * dx + dy * dy + dz * dz;
    float rinv = __builtin_amdgcn_rsqf(r2);
    float r = r2 * rinv;
    float ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
    float s = nix * ex + niy * ey + niz * ez;
    float t = njx * ex + njy * ey + njz * ez;
    float c = nix * njx + niy * njy + niz * njz;
    float a = c - s * t + st0 * (t - s) - st0 * st0;
    float phi = 1.0f + mu * (a - 1.0f);
    float U, dUdr, dUda;
    if (r < rmin) {
        float q = rmin * rmin * rinv * rinv;
        U = eps * (q * q - 2.0f * q) + (1.0f - phi) * eps;
        dUdr = 4.0f * eps * (q - q * q) * rinv;
        dUda = -mu * eps;
    } else {
        // x = (pi/2) u: the hardware sine / cosine take revolutions, x / 2pi = u / 4
        float u = (r - rmin) * inv_w;
        float sx = __builtin_amdgcn_sinf(0.25f * u);
        float cx = __builtin_amdgcn_cosf(0.25f * u);
        float c2 = cx * cx;
        float cz1 = ipow(c2, P.zeta - 1);        // cos^(2 zeta - 2)
        float uA = -eps * cz1 * c2;
        U = uA * phi;
        dUdr = phi * eps * (float)P.zeta * 3.14159265358979f * inv_w * sx * cz1 * cx;
        dUda = mu * uA;
    }
    float gx = -t * nix - s * njx + st0 * (njx - nix);
    float gy = -t * niy - s * njy + st0 * (njy - niy);
    float gz = -t * niz - s * njz + st0 * (njz - niz);
    float proj = gx * ex + gy * ey + gz * ez;
    float k = dUda * rinv;
    fx -= dUdr * ex + k * (gx - proj * ex);
    fy -= dUdr * ey + k * (gy - proj * ey);
    fz -= dUdr * ez + k * (gz - proj * ez);
    // torque on i: n_i x g_i with g_i = -dU/da (n_j - (t + sin th0) e)
    float b = t + st0;
    float wx = -dUda * (njx - b * ex), wy = -dUda * (njy - b * ey), wz = -dUda * (njz - b * ez);
    tx += niy * wz - niz * wy;
    ty += niz * wx - nix * wz;
    tz += nix * wy - niy * wx;
    return U;
}

template <>
__device__ __forceinline__ double lipid_pair<double>(const DevParams &P, double dx, double dy, double dz, double nix,
                                                     double niy, double niz, double njx, double njy, double njz,
                                                     double &fx, double &fy, double &fz, double &tx, double &ty,
                                                     double &tz) {
    const double eps = P.eps, mu = P.mu, st0 = P.st0, rmin = P.r_min, rc = P.rc_lipid;
    double r2 = dx * dx + dy * dy + dz * dz;
    double r = sqrt(r2);
    double rinv = 1.0 / r;
    double ex = dx * rinv, ey = dy * rinv, ez = dz * rinv;
    double s = nix * ex + niy * ey + niz * ez;
    double t = njx * ex + njy * ey + njz * ez;
    double c = nix * njx + niy * njy + niz * njz;
    double a = c - s * t + st0 * (t - s) - st0 * st0;
    double phi = 1.0 + mu * (a - 1.0);
    double U, dUdr, dUda;
    if (r < rmin) {
        double q = (rmin * rinv) * (rmin * rinv);
        U = eps * (q * q - 2.0 * q) + (1.0 - phi) * eps;
        dUdr = 4.0 * eps * (q - q * q) * rinv;
        dUda = -mu * eps;
    } else {
        double x = 0.5 * M_PI * (r - rmin) / (rc - rmin);
        double sx, cx;
        sincos(x, &sx, &cx);
        double c2 = cx * cx;
        double cz1 = ipow(c2, P.zeta - 1);
        double uA = -eps * cz1 * c2;
        U = uA * phi;
        dUdr = phi * eps * (double)P.zeta * M_PI / (rc - rmin) * sx * cz1 * cx;
        dUda = mu * uA;
    }
    double gx = -t * nix - s * njx + st0 * (njx - nix);
    double gy = -t * niy - s * njy + st0 * (njy - niy);
    double gz = -t * niz - s * njz + st0 * (njz - niz);
    double proj = gx * ex + gy * ey + gz * ez;
    double k = dUda * rinv;
    fx -= dUdr * ex + k * (gx - proj * ex);
    fy -= dUdr * ey + k * (gy - proj * ey);
    fz -= dUdr * ez + k * (gz - proj * ez);
    double b = t + st0;
    double wx = -dUda * (njx - b * ex), wy = -dUda * (njy - b * ey), wz = -dUda * (njz - b * ez);
    tx += niy * wz - niz * wy;
    ty += niz * wx - nix * wz;
    tz += nix * wy - niy * wx;
    return U;
}

// WCA for pairs with a protein bead; adds the force on i, returns U.
template <class T>
__device__ __forceinline__ T wca_pair(const DevParams &P, T dx, T dy, T dz, T &fx, T &fy, T &fz) {
    T r2 = dx * dx + dy * dy + dz * dz;
    T sr2 = (T)P.wca_sig2 / r2;
    T sr6 = sr2 * sr2 * sr2;
    T e = (T)P.wca_eps;
    T U = (T)4 * e * (sr6 * sr6 - sr6) + e;
    T f = (T)24 * e * ((T)2 * sr6 * sr6 - sr6) / r2;
    fx += f * dx;
    fy += f * dy;
    fz += f * dz;
    return U;
}

// ------------------------------------------------------------------ force kernel

template <int MIXED>
struct Staged;
template <>
struct Staged<1> {
    using P = D4;          // raw FP64 position, type in w (the separation is formed in FP64)
    using N = float4;      // orientation (FP32)
};
template <>
struct Staged<0> {
    using P = D4;          // raw FP64 position, type in w
    using N = D4;          // FP64 orientation
};

// One workgroup per 256 consecutive cell-sorted particles.  The block's partners
// (its stage list) are read once from HBM into LDS; lane i then walks column i of
// its chunk's list, whose entries index the LDS stage.  Every candidate takes the
// exact FP64 neighbour test on FP64 positions in both modes; mixed mode rounds the
// separation and orientations to FP32 for the pair law.
template <int MIXED, int ENERGY, int KICK>
__global__ __launch_bounds__(BLOCK) void k_force(const SysDev *Sd, Maps L_maps, DevParams P, double dt) {
    using T = typename std::conditional<MIXED, float, double>::type;
    using SP = typename Staged<MIXED>::P;
    using SN = typename Staged<MIXED>::N;
    __shared__ SP s_p[SMAX];
    __shared__ SN s_n[SMAX];
    const int s = find_sys(L_maps.p, L_maps.nsys, blockIdx.x);
    const SysDev &S = Sd[s];
    const int lb = blockIdx.x - L_maps.p[s];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int chunk = lb * (BLOCK / WAVE) + (tid >> 6);
    const int i = lb * BLOCK + tid;
    const bool valid = i < S.n;
    const int scnt = S.scount[lb];
    for (int q = tid; q < scnt; q += BLOCK) {
        const int slot = S.stage[(size_t)lb * SMAX + q];
        const D4 p = S.pos[slot];
        const D4 o = S.ori[slot];
        if constexpr (MIXED) {
            s_p[q] = p;
            s_n[q] = make_float4((float)o.x, (float)o.y, (float)o.z, 0.0f);
        } else {
            s_p[q] = p;
            s_n[q] = o;
        }
    }
    __syncthreads();
    if (chunk >= S.nchunk) return;
    const D4 pi = valid ? S.pos[i] : D4{0.0, 0.0, 0.0, 0.0};
    const D4 ni = valid ? S.ori[i] : D4{0.0, 0.0, 0.0, 0.0};
    const int ti = (int)pi.w;
    const T nix = (T)ni.x, niy = (T)ni.y, niz = (T)ni.z;
    T fx = 0, fy = 0, fz = 0, tx = 0, ty = 0, tz = 0;
    double U = 0.0, W = 0.0;
    const int rows = min(S.nlk[chunk], MAXNB);
    const int32_t *col = S.nl + (size_t)chunk * MAXNB * CHUNK + lane;
    if (scnt >= 0) {
        if constexpr (MIXED) {
            for (int r = 0; r < rows; ++r) {
                const int e = valid ? col[r * CHUNK] : -1;
                if (e < 0 || e >= scnt) continue;
                const D4 pj = s_p[e];
                const int tj = (int)pj.w;
                double dx, dy, dz;
                const double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
                if (!(d2 < P.rc2[ti][tj])) continue;
                float ax = 0.f, ay = 0.f, az = 0.f, u;
                if ((ti | tj) == 0) {
                    const float4 nj = s_n[e];
                    u = lipid_pair<float>(P, (float)dx, (float)dy, (float)dz, nix, niy, niz, nj.x, nj.y, nj.z, ax, ay,
                                          az, tx, ty, tz);
                } else {
                    u = wca_pair<float>(P, (float)dx, (float)dy, (float)dz, ax, ay, az);
                }
                fx += ax;
                fy += ay;
                fz += az;
                if (ENERGY) {
                    U += 0.5 * (double)u;
                    W += 0.5 * (dx * (double)ax + dy * (double)ay + dz * (double)az);
                }
            }
        } else {
            for (int r = 0; r < rows; ++r) {
                const int e = valid ? col[r * CHUNK] : -1;
                if (e < 0 || e >= scnt) continue;
                const D4 pj = s_p[e];
                const int tj = (int)pj.w;
                double dx, dy, dz;
                const double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
                if (!(d2 < P.rc2[ti][tj])) continue;
                double ax = 0, ay = 0, az = 0, u;
                if ((ti | tj) == 0) {
                    const D4 nj = s_n[e];
                    u = lipid_pair<double>(P, dx, dy, dz, nix, niy, niz, nj.x, nj.y, nj.z, ax, ay, az, tx, ty, tz);
                } else {
                    u = wca_pair<double>(P, dx, dy, dz, ax, ay, az);
                }
                fx += ax;
                fy += ay;
                fz += az;
                if (ENERGY) {
                    U += 0.5 * u;
                    W += 0.5 * (dx * ax + dy * ay + dz * az);
                }
            }
        }
    } else {
        // block whose partners did not fit the stage: entries are global slots
        for (int r = 0; r < rows; ++r) {
            const int j = valid ? col[r * CHUNK] : -1;
            if (j < 0 || j >= S.n) continue;
            const D4 pj = S.pos[j];
            const int tj = (int)pj.w;
            double dx, dy, dz;
            const double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
            if (!(d2 < P.rc2[ti][tj])) continue;
            T ax = 0, ay = 0, az = 0;
            T u;
            if ((ti | tj) == 0) {
                const D4 nj = S.ori[j];
                u = lipid_pair<T>(P, (T)dx, (T)dy, (T)dz, nix, niy, niz, (T)nj.x, (T)nj.y, (T)nj.z, ax, ay, az, tx,
                                  ty, tz);
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
    double Fx = (double)fx, Fy = (double)fy, Fz = (double)fz;
    D4 v = {0.0, 0.0, 0.0, 0.0}, w = {0.0, 0.0, 0.0, 0.0};
    const D4 Tq = {(double)tx, (double)ty, (double)tz, 0.0};
    if (valid) {
        // bonds of this particle (CSR by caller id), FP64 in both modes
        const int g = S.gid[i];
        for (int q = S.bstart[g]; q < S.bstart[g + 1]; ++q) {
            const int j = S.slot[S.bpart[q]];
            const D4 pj = S.pos[j];
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
        S.frc[i] = D4{Fx, Fy, Fz, 0.0};
        S.trq[i] = Tq;
        v = S.vel[i];
        w = S.angv[i];
        if (KICK) {
            const double h = 0.5 * dt * P.inv_mass[ti];
            v.x += h * Fx;
            v.y += h * Fy;
            v.z += h * Fz;
            S.vel[i] = v;
            if (ti == 0) {
                const double hw = 0.5 * dt * P.inv_inertia;
                w.x += hw * Tq.x;
                w.y += hw * Tq.y;
                w.z += hw * Tq.z;
                S.angv[i] = w;
            }
        }
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
    hipLaunchKernelGGL((k_force<MIXED, ENERGY, KICK>), dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm, dt);
}

void launch_force(const LaunchCtx &L, int mixed, int energy, int kick, double dt) {
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
    const int i = (blockIdx.x - L_maps.p[s]) * BLOCK + threadIdx.x;
    double disp2 = 0.0, v2 = 0.0;
    bool bad = false;
    if (i < S.n) {
        D4 p = S.pos[i], v = S.vel[i], f = S.frc[i];
        const int t = (int)p.w;
        const double h = 0.5 * dt * P.inv_mass[t];
        v.x += h * f.x;
        v.y += h * f.y;
        v.z += h * f.z;
        p.x += dt * v.x;
        p.y += dt * v.y;
        p.z += dt * v.z;
        S.vel[i] = v;
        S.pos[i] = p;
        if (t == 0) {
            D4 w = S.angv[i], tq = S.trq[i], n = S.ori[i];
            const double hw = 0.5 * dt * P.inv_inertia;
            w.x += hw * tq.x;
            w.y += hw * tq.y;
            w.z += hw * tq.z;
            const double wn = sqrt(w.x * w.x + w.y * w.y + w.z * w.z);
            if (wn > 0.0) {
                const double kx = w.x / wn, ky = w.y / wn, kz = w.z / wn;
                double sn, cs;
                sincos(wn * dt, &sn, &cs);
                const double kn = kx * n.x + ky * n.y + kz * n.z;
                const double cx = ky * n.z - kz * n.y, cy = kz * n.x - kx * n.z, cz = kx * n.y - ky * n.x;
                const double ox = n.x * cs + cx * sn + kx * kn * (1.0 - cs);
                const double oy = n.y * cs + cy * sn + ky * kn * (1.0 - cs);
                const double oz = n.z * cs + cz * sn + kz * kn * (1.0 - cs);
                n.x = ox; n.y = oy; n.z = oz;
            }
            const double nn = sqrt(n.x * n.x + n.y * n.y + n.z * n.z);
            if (nn > 0.0) { n.x /= nn; n.y /= nn; n.z /= nn; }
            S.angv[i] = w;
            S.ori[i] = n;
        }
        const D4 b = S.xb[i];
        const double ddx = p.x - b.x, ddy = p.y - b.y, ddz = p.z - b.z;
        disp2 = ddx * ddx + ddy * ddy + ddz * ddz;
        v2 = v.x * v.x + v.y * v.y + v.z * v.z;
        bad = !isfinite(p.x + p.y + p.z + v.x + v.y + v.z);
    }
    disp2 = wave_maxd(disp2);
    v2 = wave_maxd(v2);
    const unsigned long long anybad = __ballot(bad);
    __shared__ double s_m[2][BLOCK / WAVE];
    if (lane_id_f() == 0) {
        s_m[0][threadIdx.x >> 6] = disp2;
        s_m[1][threadIdx.x >> 6] = v2;
        if (anybad) atomicOr(&S.sc->err, ERR_NONFINITE);
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double m = s_m[threadIdx.x][0];
        for (int q = 1; q < BLOCK / WAVE; ++q) m = fmax(m, s_m[threadIdx.x][q]);
        S.bred[(size_t)(blockIdx.x - L_maps.p[s]) * BRED + threadIdx.x] = m;
    }
}

// Largest displacement since the last build and largest drift speed, per system,
// from the kick-drift block partials.
__global__ __launch_bounds__(256) void k_stats_reduce(const SysDev *Sd, int nsys) {
    const SysDev &S = Sd[blockIdx.x];
    const int nblk = (S.n + BLOCK - 1) / BLOCK;
    double d = 0.0, v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        d = fmax(d, S.bred[(size_t)b * BRED]);
        v = fmax(v, S.bred[(size_t)b * BRED + 1]);
    }
    d = wave_maxd(d);
    v = wave_maxd(v);
    __shared__ double s_m[2][4];
    if ((threadIdx.x & 63) == 0) { s_m[0][threadIdx.x >> 6] = d; s_m[1][threadIdx.x >> 6] = v; }
    __syncthreads();
    if (threadIdx.x == 0 && nblk > 0) {
        d = fmax(fmax(s_m[0][0], s_m[0][1]), fmax(s_m[0][2], s_m[0][3]));
        v = fmax(fmax(s_m[1][0], s_m[1][1]), fmax(s_m[1][2], s_m[1][3]));
        SysScal *sc = S.sc;
        if (dbits(d) > sc->maxdisp2) sc->maxdisp2 = dbits(d);
        if (dbits(v) > sc->maxv2) sc->maxv2 = dbits(v);
    }
}

void launch_kick_drift(const LaunchCtx &L, double dt) {
    hipLaunchKernelGGL(k_kick_drift, dim3(L.nblk_p), dim3(BLOCK), 0, L.st, L.S, L.maps, L.prm, dt);
    hipLaunchKernelGGL(k_stats_reduce, dim3(L.nsys), dim3(256), 0, L.st, L.S, L.nsys);
}

// ------------------------------------------------------------------ energy reduction

// Fixed-order sum of the per-chunk partials of each system (one block per system).
__global__ __launch_bounds__(256) void k_reduce_energy(const SysDev *Sd, int nsys) {
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
    if (threadIdx.x == 0)
        for (int q = 0; q < 9; ++q) S.sc->energy[q] = ((sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]));
}

void launch_reduce_energy(const LaunchCtx &L) {
    hipLaunchKernelGGL(k_reduce_energy, dim3(L.nsys), dim3(256), 0, L.st, L.S, L.nsys);
}

// ------------------------------------------------------------------ outputs in caller order

__global__ void k_scatter_state(const SysDev *Sd, int s, double *x, double *n, double *v, double *w) {
    const SysDev &S = Sd[s];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n) return;
    const int g = S.gid[i];
    if (x) { D4 p = S.pos[i]; x[3 * g] = p.x; x[3 * g + 1] = p.y; x[3 * g + 2] = p.z; }
    if (n) { D4 p = S.ori[i]; n[3 * g] = p.x; n[3 * g + 1] = p.y; n[3 * g + 2] = p.z; }
    if (v) { D4 p = S.vel[i]; v[3 * g] = p.x; v[3 * g + 1] = p.y; v[3 * g + 2] = p.z; }
    if (w) { D4 p = S.angv[i]; w[3 * g] = p.x; w[3 * g + 1] = p.y; w[3 * g + 2] = p.z; }
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
    if (F) { D4 p = S.frc[i]; F[3 * g] = p.x; F[3 * g + 1] = p.y; F[3 * g + 2] = p.z; }
    if (T) { D4 p = S.trq[i]; T[3 * g] = p.x; T[3 * g + 1] = p.y; T[3 * g + 2] = p.z; }
}

void launch_scatter_forces(const LaunchCtx &L, int sys, double *F, double *T, int count) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_scatter_forces, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, L.st, L.S, sys, F, T);
}

// ------------------------------------------------------------------ neighbour-set export

// Pairs (gid_i < gid_j) of the list that pass the exact FP64 test, appended in any
// order (one atomic per wavefront).  Staged entries are mapped back to slots.
__device__ __forceinline__ int entry_slot(const SysDev &S, int blk, int scnt, int e) {
    return scnt >= 0 ? S.stage[(size_t)blk * SMAX + e] : e;
}

__global__ void k_export_pairs(const SysDev *Sd, int s, DevParams P) {
    const SysDev &S = Sd[s];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < S.n;
    const int chunk = i / CHUNK, lane = i % CHUNK, blk = i / BLOCK;
    D4 pi = {0, 0, 0, 0};
    int ti = 0, gi = 0, rows = 0, scnt = -1;
    const int32_t *col = nullptr;
    if (valid) {
        pi = S.pos[i];
        ti = (int)pi.w;
        gi = S.gid[i];
        rows = min(S.nlk[chunk], MAXNB);
        scnt = S.scount[blk];
        col = S.nl + (size_t)chunk * MAXNB * CHUNK + lane;
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
            if (lane_id_f() == 0 && tot > 0) wb = atomicAdd(&S.sc->npairs, tot);
            base = __shfl(wb, 0) + ex;
        }
        int k = 0;
        for (int r = 0; r < rows; ++r) {
            const int e = col[r * CHUNK];
            if (e < 0) continue;
            const int j = entry_slot(S, blk, scnt, e);
            if (j < 0 || j >= S.n) continue;
            const int gj = S.gid[j];
            if (gj <= gi) continue;
            const D4 pj = S.pos[j];
            double dx, dy, dz;
            const double d2 = dist2_exact(S, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
            if (d2 < P.rc2[ti][(int)pj.w]) {
                if (pass == 1 && (int64_t)(base + k) < S.pairs_cap) {
                    S.pairs[2 * (base + k)] = gi;
                    S.pairs[2 * (base + k) + 1] = gj;
                }
                ++k;
            }
        }
        mine = k;
    }
}

void launch_export_pairs(const LaunchCtx &L, int sys, int count) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_export_pairs, dim3((count + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, L.st, L.S, sys, L.prm);
}

}  // namespace rbc
