// Host runtime of librbc: the C ABI declared in include/rbc.h.
//
// A context holds up to max_slots independent systems.  Each system owns one
// device allocation carved into its arrays; a device-side table of system
// descriptors plus block->system prefix maps lets every kernel launch serve all
// live systems at once.  The time-step loop is driven from the host with one
// step of lookahead: after each kick-drift the per-system displacement statistics
// are copied to pinned memory, and while the force kernel of step s runs the
// host decides which systems need a cell update before the force of step s+1.
// With graphs enabled (the default for ensembles) the fixed launch sequence of a
// step -- the force kernel with its fused drift and the drift statistics -- is
// captured once per system table and time step and replayed as a HIP graph; cell
// updates launch only the blocks of the systems that rebuild.
#include "../../include/rbc.h"
#include "rbc_dev.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace rbc;

namespace {

constexpr int RING = 8;
// Systems this large decide list rebuilds and prunes from the statistics of the drift to
// the current positions (exact); the margin covers the FP32 reference positions.
constexpr int64_t EXACT_MIN_N = 1 << 20;
constexpr double EXACT_MARGIN = 2e-4;

struct HostSys {
    bool live = false;
    int64_t n = 0, nlip = 0, nbond = 0;
    int64_t nsrcp = 0;               // protein beads seeding a separate cell set (0: none)
    int32_t kl = 0;                  // lipid cells; cells [kl, k) belong to the protein set
    int32_t k = 0, nchunk = 0, gcap = 0, cnbr_cap = 0, ntile_p = 0, ntile_s = 0;
    double box[3] = {0, 0, 0};
    int32_t per[3] = {0, 0, 0};
    void *mem = nullptr;
    size_t bytes = 0;
    void *pairs_mem = nullptr;
    int64_t pairs_cap = 0;
    SysDev dev{};
    int32_t *lip = nullptr;          // device: lipid ids in id order, then protein ids (the seed lists)
    int64_t steps_since = 0, steps_total = 0;
    int64_t updates = 0;             // Voronoi cell updates (each also rebuilds the lists)
    int64_t rebuilds = 0;            // neighbour-list builds of any kind
    int64_t early = 0;               // list-only rebuilds forced by the skin between cell updates
    int64_t prunes = 0;              // prunes of the lists outside a build
    bool have_stats = false, rebuilt_last = false, refreshed_last = false;
    double disp2 = 0.0, v2 = 0.0, disp2p = 0.0;
    double cur_d2 = 0.0, cur_v2 = 0.0, cur_d2p = 0.0;   // the latest drift statistics read
    uint64_t drifts = 0;             // statistics passes since loading (the device's step counter)
    bool pending = false;            // staged: uploaded, cells not built yet
    rbc_status failed = RBC_OK;      // ensemble slot frozen by an error (held until retired)
    std::string why;                 // its message
};

// A slot whose system takes part in launches: live, and not frozen by an error.
bool runs(const HostSys &hs) { return hs.live && hs.failed == RBC_OK; }

struct Carve {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
};

}  // namespace

struct rbc_ctx {
    rbc_params prm{};
    DevParams dprm{};
    hipStream_t user = nullptr, st = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int device = 0;
    int32_t max_slots = 1;
    int64_t budget = 0, used = 0;
    bool ensemble = false;
    std::vector<HostSys> sys;
    SysDev *d_sys = nullptr;
    SysScal *d_sc = nullptr;
    int32_t *d_maps = nullptr;
    int32_t *d_umaps = nullptr;       // block maps of the systems in the running cell update
    int32_t *d_pmaps = nullptr;       // particle-block map of the systems pruned at this step
    int32_t *pair_scratch = nullptr;  // this device's static staging of the allocation-free pair export
    const int32_t **d_lip = nullptr;
    SysScal *h_sc = nullptr;          // pinned mirror of the per-system scalars (read after a sync)
    StepStat *h_stat = nullptr, *d_stat = nullptr;   // published drift statistics: host / device view
    hipEvent_t step_ev[RING] = {};    // one per step in flight: the drift statistics are published
    int64_t step_pos = 0;
    LaunchCtx L{};
    int32_t nsys = 0;                 // descriptors in use (highest live slot + 1)
    bool forces_valid = false;
    bool vol_fresh = false;          // the per-chunk lipid sums describe the current state of every system
    int sticky = RBC_OK;
    std::string err;
    int64_t ens_steps = 0;
    // captured launch sequences (replayed while the system table and dt are unchanged)
    bool graphs = false;
    int64_t table_version = 0;
    int64_t graph_version = -1;
    double graph_dt = 0.0;
    hipGraphExec_t g_step = nullptr, g_last = nullptr;
    // per-step timing (events at the end of every step of a call)
    bool step_timing = false;
    std::vector<hipEvent_t> ev_step;
    hipEvent_t ev_call0 = nullptr, ev_prev_end = nullptr, ev_prev_end_last = nullptr;
    bool have_prev_end = false;
    std::vector<double> step_ms;      // the last call's step intervals
    double gap_ms = -1.0;             // from the previous call's last step to the last call's start
    // host time of the last step call, per step: outside waits for the device, and waiting
    double host_us_step = -1.0, wait_us_step = -1.0;
    // force-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> tb, te;
    int tcount = 0;
    double tsum_ms = 0.0;
    int64_t tlaunches = 0;
    // list-build kernel timing (with force timing)
    std::vector<hipEvent_t> nb, ne;
    int ncount = 0;
    double nsum_ms = 0.0;
    int64_t nlaunches = 0;
};

namespace {

rbc_status fail(rbc_ctx *h, rbc_status s, const std::string &msg) {
    if (h) h->err = msg;
    return s;
}

#define HIPCHK(call)                                                                              \
    do {                                                                                          \
        hipError_t _e = (call);                                                                   \
        if (_e != hipSuccess)                                                                     \
            return fail(h, RBC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(_e));        \
    } while (0)

struct Scope {   // orders the library stream after the caller's stream and back
    rbc_ctx *h;
    explicit Scope(rbc_ctx *hh) : h(hh) {
        hipEventRecord(h->ev_in, h->user);
        hipStreamWaitEvent(h->st, h->ev_in, 0);
    }
    ~Scope() {
        hipEventRecord(h->ev_out, h->st);
        hipStreamWaitEvent(h->user, h->ev_out, 0);
    }
};

bool valid_params(const rbc_params *p, std::string &why) {
    if (!p) { why = "params is NULL"; return false; }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (!(p->rc[a][b] > 0.0) || p->rc[a][b] != p->rc[b][a]) { why = "rc must be positive and symmetric"; return false; }
    if (!(p->r_min > 0.0) || !(p->rc[0][0] > p->r_min)) { why = "need 0 < r_min < rc[0][0]"; return false; }
    double z = p->zeta;
    if (!(z >= 1.0 && z <= 16.0) || z != std::floor(z)) { why = "zeta must be an integer in [1, 16]"; return false; }
    for (int a = 0; a < 3; ++a) if (!(p->mass[a] > 0.0)) { why = "masses must be positive"; return false; }
    if (!(p->inertia > 0.0)) { why = "inertia must be positive"; return false; }
    if (p->cell_target < 1) { why = "cell_target must be >= 1"; return false; }
    if (p->update_every < 1) { why = "update_every must be >= 1"; return false; }
    if (!(p->skin >= 0.0)) { why = "skin must be >= 0"; return false; }
    if (p->lloyd_iters < 1) { why = "lloyd_iters must be >= 1"; return false; }
    if (p->precision != RBC_FP64 && p->precision != RBC_MIXED) { why = "unknown precision"; return false; }
    if (p->protein_cells != 0 && p->protein_cells != 1) { why = "protein_cells must be 0 or 1"; return false; }
    if (!(p->vol_k >= 0.0) || !(p->vol_target >= 0.0)) { why = "vol_k and vol_target must be >= 0"; return false; }
    if (p->vol_k > 0.0 && !(p->lipid_area > 0.0)) { why = "the volume constraint needs lipid_area > 0"; return false; }
    if (!(p->kT >= 0.0) || !(p->gamma >= 0.0) || !(p->gamma_rot >= 0.0)) { why = "kT, gamma and gamma_rot must be >= 0"; return false; }
    if (p->quench != 0 && p->quench != 1) { why = "quench must be 0 or 1"; return false; }
    if (p->quench && !(p->quench_max > 0.0)) { why = "quenching needs quench_max > 0"; return false; }
    if (p->quench && (p->gamma > 0.0 || p->gamma_rot > 0.0)) { why = "quenching excludes the thermostat"; return false; }
    if (!(p->wca_sigma > 0.0) || !(p->k_bond >= 0.0)) { why = "bad WCA / bond constants"; return false; }
    return true;
}

// Half-width of the pruned lists' buffer: params.inner_skin, or the full skin when
// that is not in (0, skin) (the lists are then pruned only when they are built).
double inner_skin(const rbc_params &p) {
    return (p.inner_skin > 0.0 && p.inner_skin < p.skin) ? p.inner_skin : p.skin;
}

void make_dev_params(rbc_ctx *h) {
    const rbc_params &p = h->prm;
    DevParams &d = h->dprm;
    double search = 0.0;
    for (int a = 0; a < 3; ++a) {
        double m = 0.0;
        for (int b = 0; b < 3; ++b) m = std::max(m, p.rc[a][b] + 2.0 * p.skin + 1e-3);
        d.rlmaxf[a] = std::nextafter((float)m, INFINITY);
    }
    const double din = inner_skin(p);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            d.rc2[a][b] = p.rc[a][b] * p.rc[a][b];
            double rl = p.rc[a][b] + 2.0 * p.skin;
            d.rl2[a][b] = rl * rl * (1.0 + 1e-12);
            d.rl2f[a][b] = std::nextafter((float)((rl + 1e-3) * (rl + 1e-3)), INFINITY);
            const double ri = p.rc[a][b] + 2.0 * din + 1e-3;
            d.rin2f[a][b] = std::nextafter((float)(ri * ri), INFINITY);
            // the FP32 square of the FP32-rounded separation is within a relative 4e-7 of
            // the exact square; a band ten times wider goes to the FP64 test
            d.rc2lo[a][b] = std::nextafter((float)(d.rc2[a][b] * (1.0 - 4e-6)), 0.0f);
            d.rc2hi[a][b] = std::nextafter((float)(d.rc2[a][b] * (1.0 + 4e-6)), INFINITY);
            search = std::max(search, rl);
        }
    d.rc_lipid = p.rc[0][0];
    d.r_min = p.r_min;
    d.eps = p.eps;
    d.mu = p.mu;
    d.st0 = p.sin_theta0;
    d.wca_eps = p.wca_eps;
    d.wca_sig2 = p.wca_sigma * p.wca_sigma;
    d.k_bond = p.k_bond;
    for (int a = 0; a < 3; ++a) d.inv_mass[a] = 1.0 / p.mass[a];
    d.inv_inertia = 1.0 / p.inertia;
    d.cell_search = search;
    d.zeta = (int32_t)p.zeta;
    d.inv_w = 1.0 / (p.rc[0][0] - p.r_min);
    d.dudr_k = p.eps * p.zeta * M_PI / (p.rc[0][0] - p.r_min);
    d.vol_on = p.vol_k > 0.0;
    d.vol_k = p.vol_k;
    d.vol_target = p.vol_target;
    d.vol_a3 = p.lipid_area / 3.0;
    d.thermo_on = p.gamma > 0.0 || p.gamma_rot > 0.0;
    d.seed_lo = (uint32_t)p.seed;
    d.seed_hi = (uint32_t)(p.seed >> 32);
    d.ou_c = d.ou_cr = 1.0;
    d.ou_a[0] = d.ou_a[1] = d.ou_a[2] = d.ou_ar = 0.0;
    d.quench_on = p.quench;
    d.quench_max = p.quench_max;
}

// Thermostat coefficients for time step dt: the exact Ornstein-Uhlenbeck decay
// c = exp(-gamma dt) and the noise amplitude per centred Philox word,
// sqrt((1 - c^2) kT / m) sqrt(12) / 2^32 (unit variance per component).
void set_step_dt(rbc_ctx *h, double dt) {
    DevParams &d = h->dprm;
    const rbc_params &p = h->prm;
    const double unit = std::sqrt(12.0) / 4294967296.0;
    d.ou_c = p.gamma > 0.0 ? std::exp(-p.gamma * dt) : 1.0;
    for (int t = 0; t < 3; ++t) d.ou_a[t] = std::sqrt((1.0 - d.ou_c * d.ou_c) * p.kT / p.mass[t]) * unit;
    d.ou_cr = p.gamma_rot > 0.0 ? std::exp(-p.gamma_rot * dt) : 1.0;
    d.ou_ar = std::sqrt((1.0 - d.ou_cr * d.ou_cr) * p.kT / p.inertia) * unit;
    h->L.prm = d;
}

// Sizes of one system and (with base != null) its device layout.
size_t layout(HostSys &s, char *base) {
    Carve c{base};
    const int64_t n = s.n;
    const int32_t k = s.k;
    SysDev &d = s.dev;
    d.pos = c.take<V3>(n); d.vel = c.take<V3>(n); d.ori = c.take<V3>(n); d.angv = c.take<V3>(n);
    d.frc = c.take<V3>(n); d.trq = c.take<V3>(n); d.xb = c.take<F3>(n); d.xp = c.take<F3>(n);
    d.pos2 = c.take<V3>(n); d.vel2 = c.take<V3>(n); d.ori2 = c.take<V3>(n); d.angv2 = c.take<V3>(n);
    d.gid = c.take<int32_t>(n); d.gid2 = c.take<int32_t>(n); d.slot = c.take<int32_t>(n);
    d.owner = c.take<int32_t>(n);
    d.key = c.take<uint64_t>(n); d.key2 = c.take<uint64_t>(n);
    d.val = c.take<uint32_t>(n); d.val2 = c.take<uint32_t>(n);
    d.hist = c.take<int32_t>((size_t)256 * (std::max(s.ntile_p, s.ntile_s) + 1));   // + digit totals
    d.seed = c.take<D4>(k); d.seed2 = c.take<D4>(k);
    d.sbox = c.take<double>((size_t)((k + BLOCK - 1) / BLOCK) * 6);
    d.cstart = c.take<int32_t>(k + 1); d.ccount = c.take<int32_t>(k); d.cstart2 = c.take<int32_t>(k + 1);
    d.ccount2 = c.take<int32_t>(k); d.cmap = c.take<int32_t>(k);
    d.cnbr_start = c.take<int32_t>(k + 1); d.cnbr = c.take<int32_t>(s.cnbr_cap);
    d.gstart = c.take<int32_t>(s.gcap + 1); d.gcount = c.take<int32_t>(s.gcap);
    d.gseed = c.take<int32_t>(k); d.sgcell = c.take<int32_t>(k);
    d.gpos = c.take<D4>(k);
    d.nl = c.take<int32_t>((size_t)s.nchunk * MAXNB * CHUNK); d.nlk = c.take<int32_t>(s.nchunk);
    d.nl16 = c.take<uint16_t>((size_t)s.nchunk * MAXNB * CHUNK);
    d.typ = c.take<uint8_t>(n); d.typ2 = c.take<uint8_t>(n);
    d.ori32 = c.take<F4>(n);
    d.ori32b = c.take<F4>(n);
    d.bstart = c.take<int32_t>(n + 1); d.bpart = c.take<int32_t>(2 * s.nbond); d.br0 = c.take<double>(2 * s.nbond);
    d.epart = c.take<double>((size_t)s.nchunk * 9);
    d.vpart = c.take<double>((size_t)s.nchunk * 8);
    d.vred = c.take<double>(32 * 8);
    const int64_t nblkp = (n + BLOCK - 1) / BLOCK;
    d.stage = c.take<int32_t>((size_t)nblkp * SSTRIDE);
    d.scount = c.take<int32_t>(nblkp);
    d.il16 = c.take<uint16_t>((size_t)s.nchunk * MAXNB * CHUNK + 16 * CHUNK);   // + rows the step kernel may prefetch
    d.ilk = c.take<int32_t>(s.nchunk);
    d.istage = c.take<int32_t>((size_t)nblkp * SSTRIDE);
    d.iscount = c.take<int32_t>(nblkp);
    d.bred = c.take<double>((size_t)nblkp * BRED);
    d.tsum = c.take<int32_t>((size_t)std::max((k + SCAN_TILE - 1) / SCAN_TILE, (s.gcap + SCAN_TILE - 1) / SCAN_TILE) + 2);
    s.lip = c.take<int32_t>(s.nlip + s.nsrcp);
    return c.off + 256;
}

void size_system(const rbc_ctx *h, HostSys &s, int64_t n, int64_t nlip, int64_t nbond) {
    s.n = n;
    s.nlip = nlip > 0 ? nlip : n;
    s.nbond = nbond;
    const int64_t m = h->prm.cell_target;
    const int64_t kl = std::max<int64_t>(1, (s.nlip + m - 1) / m);
    // a separate protein cell set needs lipids and proteins both
    s.nsrcp = (h->prm.protein_cells && nlip > 0 && n > nlip) ? n - nlip : 0;
    s.kl = (int32_t)kl;
    s.k = (int32_t)(kl + (s.nsrcp + m - 1) / m);
    s.nchunk = (int32_t)((n + CHUNK - 1) / CHUNK);
    s.gcap = 8 * s.k + 64;
    s.cnbr_cap = 96 * s.k + 1024;
    s.ntile_p = (int32_t)((n + SORT_TILE - 1) / SORT_TILE);
    s.ntile_s = (s.k + SORT_TILE - 1) / SORT_TILE;
}

int key_bits(int32_t k) {
    int b = 1;
    while ((1ll << b) < (int64_t)k) ++b;
    return b;
}

// Rebuild the device descriptor table and the block maps after a membership change.
rbc_status refresh_tables(rbc_ctx *h) {
    int top = 0;
    for (int s = 0; s < h->max_slots; ++s)
        if (h->sys[s].live) top = s + 1;
    h->nsys = std::max(top, 1);
    // frozen slots keep their memory but get an empty descriptor: no kernel touches them
    const int ns = h->nsys;
    std::vector<SysDev> tab(ns);
    std::vector<const int32_t *> lips(ns, nullptr);
    std::vector<int32_t> maps(8 * (ns + 1), 0);
    int32_t kmin = INT32_MAX, kmax = 0;
    int32_t *mp = maps.data(), *mc = mp + (ns + 1), *mg = mc + (ns + 1), *mtp = mg + (ns + 1), *mts = mtp + (ns + 1);
    int32_t *msc = mts + (ns + 1), *msg = msc + (ns + 1), *mf = msg + (ns + 1);
    for (int s = 0; s < ns; ++s) {
        HostSys &hs = h->sys[s];
        SysDev d{};
        if (runs(hs)) {
            d = hs.dev;
            lips[s] = hs.lip;
        }
        d.sc = h->d_sc + s;
        d.hstat = h->d_stat + (size_t)s * STAT_RING;
        tab[s] = d;
        const bool on = runs(hs);
        const int64_t n = on ? hs.n : 0;
        const int32_t k = on ? hs.k : 0;
        if (on) { kmin = std::min(kmin, k); kmax = std::max(kmax, k); }
        mp[s + 1] = mp[s] + (int32_t)((n + BLOCK - 1) / BLOCK);
        mc[s + 1] = mc[s] + (k + BLOCK - 1) / BLOCK;
        mg[s + 1] = mg[s] + (on ? (hs.gcap + BLOCK - 1) / BLOCK : 0);
        mtp[s + 1] = mtp[s] + (on ? hs.ntile_p : 0);
        mts[s + 1] = mts[s] + (on ? hs.ntile_s : 0);
        msc[s + 1] = msc[s] + (k + SCAN_TILE - 1) / SCAN_TILE;
        msg[s + 1] = msg[s] + (on ? (hs.gcap + SCAN_TILE - 1) / SCAN_TILE : 0);
        mf[s + 1] = mf[s] + (mp[s + 1] - mp[s]) * (d.split ? 4 : 1);
    }
    HIPCHK(hipMemcpyAsync(h->d_sys, tab.data(), sizeof(SysDev) * ns, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemcpyAsync(h->d_maps, maps.data(), sizeof(int32_t) * maps.size(), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipMemcpyAsync(h->d_lip, lips.data(), sizeof(void *) * ns, hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));   // host staging vectors go out of scope
    h->table_version++;
    LaunchCtx &L = h->L;
    L.S = h->d_sys;
    L.Sw = h->d_sys;
    L.maps.p = h->d_maps;
    L.maps.c = h->d_maps + (ns + 1);
    L.maps.g = h->d_maps + 2 * (ns + 1);
    L.maps.tp = h->d_maps + 3 * (ns + 1);
    L.maps.ts = h->d_maps + 4 * (ns + 1);
    L.maps.sc = h->d_maps + 5 * (ns + 1);
    L.maps.sg = h->d_maps + 6 * (ns + 1);
    L.maps.f = h->d_maps + 7 * (ns + 1);
    L.maps.nsys = ns;
    L.kmin = kmin;
    L.kmax = kmax;
    L.nblk_p = mp[ns];
    L.nblk_c = mc[ns];
    L.nblk_g = mg[ns];
    L.nblk_tp = mtp[ns];
    L.nblk_ts = mts[ns];
    L.nblk_sc = msc[ns];
    L.nblk_sg = msg[ns];
    L.nblk_f = mf[ns];
    L.nsys = ns;
    L.prm = h->dprm;
    L.st = h->st;
    return RBC_OK;
}

bool any_live(const rbc_ctx *h) {
    for (const auto &s : h->sys)
        if (runs(s)) return true;
    return false;
}

void update_body(rbc_ctx *h, const LaunchCtx &L, int bits, int lloyd);
void lists_body(rbc_ctx *h, const LaunchCtx &L, bool cells_moved);

// Launch context whose block maps cover only the systems in `which`, with their
// rebuild flags set: the device builds the restricted prefix maps from the flags,
// the host sums the same block counts for the grid sizes.
LaunchCtx restricted(rbc_ctx *h, const std::vector<int> &which) {
    unsigned long long m[4] = {0, 0, 0, 0};
    for (int s : which) m[s >> 6] |= 1ull << (s & 63);
    const LaunchCtx &L = h->L;
    launch_set_rebuild(L, m);
    launch_restrict_maps(L, h->d_umaps);
    LaunchCtx U = L;
    const int ns = h->nsys;
    U.maps.p = h->d_umaps;
    U.maps.c = h->d_umaps + (ns + 1);
    U.maps.g = h->d_umaps + 2 * (ns + 1);
    U.maps.tp = h->d_umaps + 3 * (ns + 1);
    U.maps.ts = h->d_umaps + 4 * (ns + 1);
    U.maps.sc = h->d_umaps + 5 * (ns + 1);
    U.maps.sg = h->d_umaps + 6 * (ns + 1);
    U.nblk_p = U.nblk_c = U.nblk_g = U.nblk_tp = U.nblk_ts = U.nblk_sc = U.nblk_sg = 0;
    U.kmin = INT32_MAX;
    U.kmax = 0;
    for (int s : which) {
        const HostSys &hs = h->sys[s];
        U.kmin = std::min(U.kmin, hs.k);
        U.kmax = std::max(U.kmax, hs.k);
        U.nblk_p += (int32_t)((hs.n + BLOCK - 1) / BLOCK);
        U.nblk_c += (hs.k + BLOCK - 1) / BLOCK;
        U.nblk_g += (hs.gcap + BLOCK - 1) / BLOCK;
        U.nblk_tp += hs.ntile_p;
        U.nblk_ts += hs.ntile_s;
        U.nblk_sc += (hs.k + SCAN_TILE - 1) / SCAN_TILE;
        U.nblk_sg += (hs.gcap + SCAN_TILE - 1) / SCAN_TILE;
    }
    return U;
}

// Run the cell update for the systems in `which`.  lloyd > 0: seed from lipids and
// run that many k-means iterations first.
void run_update(rbc_ctx *h, const std::vector<int> &which, int lloyd) {
    if (which.empty()) return;
    int32_t kmax = 1;
    for (int s : which) kmax = std::max(kmax, h->sys[s].k);
    const LaunchCtx U = restricted(h, which);
    update_body(h, U, key_bits(kmax), lloyd);
    for (int s : which) {
        HostSys &hs = h->sys[s];
        hs.updates++;
        hs.rebuilds++;
        hs.steps_since = 0;
    }
}

// Rebuild only the neighbour lists of the systems in `which`, on their current
// cells: particles keep their cells, whose radii grow to the members' current
// distances, so the cell pairs and the lists stay complete.
void run_lists(rbc_ctx *h, const std::vector<int> &which) {
    if (which.empty()) return;
    lists_body(h, restricted(h, which), false);
    for (int s : which) h->sys[s].rebuilds++;
}

// Prune the lists of the systems in `which` at their current positions (their lists
// stay as built).  When every live system prunes, the full particle map serves.
void run_prunes(rbc_ctx *h, const std::vector<int> &which) {
    if (which.empty()) return;
    LaunchCtx P = h->L;
    int live = 0;
    for (const auto &hs : h->sys) live += hs.live;
    if ((int)which.size() != live) {
        unsigned long long m[4] = {0, 0, 0, 0};
        P.nblk_p = 0;
        for (int s : which) {
            m[s >> 6] |= 1ull << (s & 63);
            P.nblk_p += (int32_t)((h->sys[s].n + BLOCK - 1) / BLOCK);
        }
        launch_mask_maps(h->L, m, h->d_pmaps);
        P.maps.p = h->d_pmaps;
    }
    launch_prune(P);
    for (int s : which) h->sys[s].prunes++;
}

// The cell-update launches for the systems whose rebuild flag is set (L carries
// block maps restricted to them).
void update_body(rbc_ctx *h, const LaunchCtx &L, int bits, int lloyd) {
    auto estep_msteps = [&](int iters) {
        for (int it = 0; it < iters; ++it) {
            if (it > 0) launch_grid_build(L);
            launch_assign(L, 1);
            launch_sort_particles(L, bits);
            launch_gather_particles(L, it == iters - 1);   // the update swaps buffers exactly twice
            launch_cell_ranges(L);
            launch_mstep(L);
        }
    };
    if (lloyd > 0) {
        launch_init_seeds(L, h->d_lip);
        launch_grid_build(L);
        estep_msteps(lloyd);
    } else {
        estep_msteps(1);    // the seed grid of the current centroids is still valid
    }
    launch_morton_sort_seeds(L);
    launch_block_permute(L);
    launch_grid_build(L);
    lists_body(h, L, true);
}

// Cell radii, cell pairs and neighbour lists on the current cells.
void lists_body(rbc_ctx *h, const LaunchCtx &L, bool cells_moved) {
    launch_cell_bounds(L);
    launch_cell_pairs(L);
    const bool t = h->timing && h->ncount < (int)h->nb.size();
    if (t) hipEventRecord(h->nb[h->ncount], L.st);
    launch_nlist(L);
    if (t) hipEventRecord(h->ne[h->ncount++], L.st);
    launch_finish_update(L, cells_moved);
}

// The status and message of one slot's error bits.
rbc_status slot_error(rbc_ctx *h, int s, int e) {
    if (e & ERR_NONFINITE) return fail(h, RBC_ERR_NONFINITE, "non-finite positions or velocities in slot " + std::to_string(s));
    if (e & ERR_NLIST) return fail(h, RBC_ERR_CAPACITY, "a particle has more than " + std::to_string(MAXNB) + " neighbours within rc + 2 skin (slot " + std::to_string(s) + ")");
    if (e & ERR_CNBR) return fail(h, RBC_ERR_CAPACITY, "cell-pair list capacity exceeded (slot " + std::to_string(s) + ")");
    if (e & ERR_ASSIGN) return fail(h, RBC_ERR_CAPACITY, "nearest-seed search failed (slot " + std::to_string(s) + ")");
    return RBC_OK;
}

rbc_status read_errors(rbc_ctx *h, const SysScal *sc) {
    for (int s = 0; s < h->nsys; ++s) {
        if (!runs(h->sys[s])) continue;
        const rbc_status r = slot_error(h, s, sc[s].err);
        if (r != RBC_OK) return r;
    }
    return RBC_OK;
}

// Ensemble contexts: after a synchronised step call, every slot whose error bits are set
// (or that the host loop found in error) is frozen -- it keeps its memory and its slot
// but leaves every launch -- so that the other slots go on.  Returns the first status.
rbc_status freeze_failed(rbc_ctx *h, const std::vector<std::pair<int, std::string>> &host_err) {
    rbc_status first = RBC_OK;
    std::string first_why;
    bool changed = false;
    auto freeze = [&](int s, rbc_status r, const std::string &why) {
        HostSys &hs = h->sys[s];
        if (!runs(hs)) return;
        hs.failed = r;
        hs.why = why;
        changed = true;
        if (first == RBC_OK) { first = r; first_why = why; }
    };
    for (int s = 0; s < h->nsys; ++s) {
        if (!runs(h->sys[s])) continue;
        const rbc_status r = slot_error(h, s, h->h_sc[s].err);
        if (r != RBC_OK) freeze(s, r, h->err);
    }
    for (const auto &e : host_err) freeze(e.first, RBC_ERR_SKIN, e.second);
    if (changed) refresh_tables(h);
    if (first != RBC_OK) h->err = first_why;
    return first;
}

bool any_pending(const rbc_ctx *h) {
    for (const auto &hs : h->sys)
        if (hs.live && hs.pending) return true;
    return false;
}

rbc_status sync_and_check(rbc_ctx *h) {
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return fail(h, RBC_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(le));
    HIPCHK(hipMemcpyAsync(h->h_sc, h->d_sc, sizeof(SysScal) * h->nsys, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return read_errors(h, h->h_sc);
}

void force_launch(rbc_ctx *h, int energy, int kick, double dt) {
    if (h->dprm.vol_on && !h->vol_fresh) {
        launch_volume_partials(h->L);   // no drift has produced them since loading
        h->vol_fresh = true;
    }
    const bool t = h->timing && h->tcount < (int)h->tb.size();
    if (t) hipEventRecord(h->tb[h->tcount], h->st);
    launch_force(h->L, h->prm.precision == RBC_MIXED, energy, kick, dt);
    if (t) {
        hipEventRecord(h->te[h->tcount], h->st);
        h->tcount++;
    }
}

void harvest_timing(rbc_ctx *h) {
    for (int q = 0; q < h->tcount; ++q) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->tb[q], h->te[q]) == hipSuccess) {
            h->tsum_ms += ms;
            h->tlaunches++;
        }
    }
    h->tcount = 0;
    for (int q = 0; q < h->ncount; ++q) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->nb[q], h->ne[q]) == hipSuccess) {
            h->nsum_ms += ms;
            h->nlaunches++;
        }
    }
    h->ncount = 0;
}

rbc_status ensure_forces(rbc_ctx *h) {
    if (!h->forces_valid) {
        force_launch(h, 0, 0, 0.0);
        h->forces_valid = true;
    }
    return RBC_OK;
}

void drop_graphs(rbc_ctx *h) {
    for (hipGraphExec_t *g : {&h->g_step, &h->g_last})
        if (*g) {
            hipGraphExecDestroy(*g);
            *g = nullptr;
        }
    h->graph_version = -1;
}

// Whether some running system needs the statistics kernel after a fused drift (small,
// split systems publish their statistics from the step kernel).
bool stats_kernel_needed(const rbc_ctx *h) {
    for (int s = 0; s < h->nsys; ++s) {
        const HostSys &hs = h->sys[s];
        if (runs(hs) && hs.n > 0 && !hs.dev.split) return true;
    }
    return false;
}

template <class F>
hipGraphExec_t capture(rbc_ctx *h, F body) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    if (hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    body();
    if (hipStreamEndCapture(h->st, &g) != hipSuccess || !g) return nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
    hipGraphDestroy(g);
    return ex;
}

// Capture the step sequences for the current table and dt.  Returns false (eager
// launches are used) if capture fails.
bool ensure_graphs(rbc_ctx *h, double dt) {
    if (h->graph_version == h->table_version && h->graph_dt == dt && h->g_step && h->g_last) return true;
    drop_graphs(h);
    const int mixed = h->prm.precision == RBC_MIXED;
    const bool stats = stats_kernel_needed(h);
    h->g_step = capture(h, [&] {
        launch_force(h->L, mixed, 0, 2, dt);
        if (stats) launch_drift_stats_swap(h->L);
    });
    h->g_last = capture(h, [&] { launch_force(h->L, mixed, 0, 1, dt); });
    if (!(h->g_step && h->g_last)) {
        drop_graphs(h);
        hipGetLastError();
        return false;
    }
    h->graph_version = h->table_version;
    h->graph_dt = dt;
    return true;
}

// The drift of every step but the first is fused into the previous step's force
// kernel, which wrote the second position / orientation buffers; the statistics
// kernel swaps them in on the device, and the host mirror follows.
void swap_drift_buffers(rbc_ctx *h) {
    for (auto &hs : h->sys)
        if (hs.live) {
            std::swap(hs.dev.pos, hs.dev.pos2);
            std::swap(hs.dev.ori, hs.dev.ori2);
            std::swap(hs.dev.ori32, hs.dev.ori32b);
        }
}

// The time-step loop over every live system.
rbc_status step_all(rbc_ctx *h, int64_t nsteps, double dt) {
    if (!any_live(h)) return RBC_OK;
    if (nsteps <= 0) return RBC_OK;
    set_step_dt(h, dt);
    const bool graphs = h->graphs && !h->timing && ensure_graphs(h, dt);
    ensure_forces(h);
    const double skin = h->prm.skin;
    const double din = inner_skin(h->prm);
    const int64_t K = h->prm.update_every;
    rbc_status out = RBC_OK;
    std::vector<std::pair<int, std::string>> slot_err;   // ensembles: per-slot errors of the host loop
    auto host_fail = [&](int s, rbc_status r, const std::string &msg) {
        if (h->ensemble) slot_err.emplace_back(s, msg);
        else if (out == RBC_OK) out = fail(h, r, msg);
    };
    const bool timed = h->step_timing;
    if (timed) {
        while ((int64_t)h->ev_step.size() < nsteps) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return fail(h, RBC_ERR_HIP, "hipEventCreate");
            h->ev_step.push_back(e);
        }
        hipEventRecord(h->ev_call0, h->st);
    }
    const bool stats_kernel = stats_kernel_needed(h);
    bool exact_any = false;
    for (const auto &hs : h->sys)
        if (runs(hs) && hs.n >= EXACT_MIN_N) exact_any = true;
    // the statistics of the latest drift of every running system, from the pinned ring
    auto read_stats = [&]() {
        for (int s = 0; s < h->nsys; ++s) {
            HostSys &hs = h->sys[s];
            if (!runs(hs)) continue;
            hs.cur_d2 = hs.cur_v2 = hs.cur_d2p = 0.0;
            if (hs.n == 0) continue;
            const volatile StepStat &e = h->h_stat[(size_t)s * STAT_RING + hs.drifts % STAT_RING];
            if (e.tag != hs.drifts + 1 && out == RBC_OK)
                out = fail(h, RBC_ERR_HIP, "drift statistics out of sequence (slot " + std::to_string(s) + ")");
            hs.cur_d2 = e.d2;
            hs.cur_v2 = e.v2;
            hs.cur_d2p = e.d2p;
            hs.drifts++;
        }
    };
    using clk = std::chrono::steady_clock;
    const auto t_loop0 = clk::now();
    double wait_s = 0.0;
    // Waiting for a step's drift statistics: poll the ring tags in pinned memory (the
    // device writes them last, after a system-scope fence), checking the event that
    // follows their publication every 64 polls; the event completing (or failing) ends
    // the wait too, and read_stats then checks the tags.  Polling answers within about
    // a microsecond of the publication, where a blocking event wait takes several.
    auto stats_ready = [&]() {
        for (int s = 0; s < h->nsys; ++s) {
            const HostSys &hs = h->sys[s];
            if (!runs(hs) || hs.n == 0) continue;
            const volatile StepStat &e = h->h_stat[(size_t)s * STAT_RING + hs.drifts % STAT_RING];
            if (e.tag != hs.drifts + 1) return false;
        }
        return true;
    };
    auto wait_event = [&](hipEvent_t ev) {
        const auto a = clk::now();
        for (int k = 1;; ++k) {
            if (stats_ready()) break;
            if (k % 64 == 0 && hipEventQuery(ev) != hipErrorNotReady) break;
        }
        wait_s += std::chrono::duration<double>(clk::now() - a).count();
    };
    launch_kick_drift(h->L, dt);
    h->vol_fresh = true;              // every drift also writes the volume's lipid sums
    for (int64_t st = 0; st < nsteps; ++st) {
        const bool last = st + 1 == nsteps;
        const int slot = (int)(h->step_pos % RING);
        h->step_pos++;
        // the statistics of the drift to this step's positions are published when
        // this event completes
        hipEventRecord(h->step_ev[slot], h->st);
        // Systems of at least EXACT_MIN_N particles decide from the statistics of the drift
        // to this step's positions.  The host waits for them (the GPU idles for the host's
        // reaction time) only when the previous step's statistics plus a bound on one more
        // drift cannot rule out a prune; otherwise no list work is due and nothing waits.
        // Smaller systems always decide from the previous step's statistics plus that bound,
        // while this step's force runs.  A system's rule depends on its own size and
        // statistics only, so its trajectory does not depend on its batch.
        bool waited = false;
        if (exact_any) {
            bool need = false;
            for (const auto &hs : h->sys) {
                if (!runs(hs) || hs.n < EXACT_MIN_N || hs.steps_since + 1 >= K) continue;
                if (!hs.have_stats) { need = true; break; }
                const double pred_p = (hs.refreshed_last ? 0.0 : std::sqrt(hs.disp2p)) + 2.0 * dt * std::sqrt(hs.v2);
                if (pred_p > din - EXACT_MARGIN) { need = true; break; }
            }
            if (need) {
                wait_event(h->step_ev[slot]);
                read_stats();
                waited = true;
            }
        }
        // decide which systems update their cells (every K steps), which rebuild their
        // lists (the skin is running out) and which prune them (the pruned lists' buffer
        // is running out; a prune needs the full lists to still hold every pair within
        // the pruned radius)
        std::vector<int> which, full, lists, pruned;
        for (int s = 0; s < h->nsys; ++s) {
            HostSys &hs = h->sys[s];
            if (!runs(hs)) continue;
            hs.steps_since++;
            if (hs.steps_since >= K) {
                full.push_back(s);
                which.push_back(s);
                continue;
            }
            bool prune = false, rebuild = false;
            if (hs.n >= EXACT_MIN_N) {
                // exact displacements at this step's positions (FP32 references: margin);
                // without them the bound above has ruled out any list work
                if (waited && std::sqrt(hs.cur_d2p) > din - EXACT_MARGIN) {
                    prune = true;
                    rebuild = std::sqrt(hs.cur_d2) > skin - din - EXACT_MARGIN;
                }
            } else if (hs.have_stats) {
                const double step_max = 2.0 * dt * std::sqrt(hs.v2);
                const double pred_p = (hs.refreshed_last ? 0.0 : std::sqrt(hs.disp2p)) + step_max;
                if (pred_p > 0.9 * din) {
                    prune = true;
                    const double pred_b = (hs.rebuilt_last ? 0.0 : std::sqrt(hs.disp2)) + step_max;
                    rebuild = pred_b > 0.9 * (skin - din);
                }
            }
            if (rebuild) {
                hs.early++;
                lists.push_back(s);
                which.push_back(s);
            } else if (prune) {
                pruned.push_back(s);
            }
        }
        run_update(h, full, 0);
        run_lists(h, lists);
        run_prunes(h, pruned);
        if (graphs) {
            hipGraphLaunch(last ? h->g_last : h->g_step, h->st);
        } else {
            force_launch(h, 0, last ? 1 : 2, dt);
            if (!last && stats_kernel) launch_drift_stats_swap(h->L);
        }
        if (!last) swap_drift_buffers(h);
        if (timed) hipEventRecord(h->ev_step[st], h->st);
        // while the force runs, read this step's drift statistics (unless read above)
        if (!waited) {
            wait_event(h->step_ev[slot]);
            read_stats();
        }
        for (int s = 0; s < h->nsys; ++s) {
            HostSys &hs = h->sys[s];
            if (!runs(hs)) continue;
            const bool rebuilt = std::find(which.begin(), which.end(), s) != which.end();
            const bool was_pruned = std::find(pruned.begin(), pruned.end(), s) != pruned.end();
            const double d2 = hs.cur_d2, v2 = hs.cur_v2, d2p = hs.cur_d2p;
            // the force of this step walked the pruned lists: they had to hold every pair in
            // range, and a prune at this step needed the full lists to hold its radius
            if (!rebuilt && !was_pruned && d2p > din * din)
                host_fail(s, RBC_ERR_SKIN, "a particle moved beyond the pruned lists' buffer before they were pruned again (slot " + std::to_string(s) + ")");
            if (was_pruned && d2 > (skin - din) * (skin - din))
                host_fail(s, RBC_ERR_SKIN, "a particle moved beyond the skin before its lists were rebuilt (slot " + std::to_string(s) + ")");
            hs.disp2 = d2;
            hs.disp2p = d2p;
            hs.v2 = std::max(v2, hs.rebuilt_last ? 0.0 : hs.v2);
            hs.have_stats = true;
            hs.rebuilt_last = rebuilt;
            hs.refreshed_last = rebuilt || was_pruned;
            hs.steps_total++;
        }
        if (h->timing && h->tcount >= (int)h->tb.size()) {   // the timing events are all in use
            const auto a = clk::now();
            HIPCHK(hipStreamSynchronize(h->st));
            wait_s += std::chrono::duration<double>(clk::now() - a).count();
            harvest_timing(h);
        }
    }
    {
        const double loop_s = std::chrono::duration<double>(clk::now() - t_loop0).count();
        h->host_us_step = (loop_s - wait_s) / (double)nsteps * 1e6;
        h->wait_us_step = wait_s / (double)nsteps * 1e6;
    }
    h->ens_steps += nsteps;
    if (timed) hipEventRecord(h->ev_prev_end, h->st);
    rbc_status e;
    if (h->ensemble) {
        // one slot's error freezes that slot only; the others have advanced nsteps
        hipError_t le = hipGetLastError();
        if (le != hipSuccess) return fail(h, RBC_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(le));
        HIPCHK(hipMemcpyAsync(h->h_sc, h->d_sc, sizeof(SysScal) * h->nsys, hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        e = freeze_failed(h, slot_err);
    } else {
        e = sync_and_check(h);
    }
    harvest_timing(h);
    if (timed) {
        h->step_ms.assign((size_t)nsteps, 0.0);
        for (int64_t st = 0; st < nsteps; ++st) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, st == 0 ? h->ev_call0 : h->ev_step[st - 1], h->ev_step[st]);
            h->step_ms[st] = ms;
        }
        float gap = -1.f;
        if (h->have_prev_end && hipEventElapsedTime(&gap, h->ev_prev_end_last, h->ev_call0) != hipSuccess) gap = -1.f;
        h->gap_ms = gap;
        std::swap(h->ev_prev_end, h->ev_prev_end_last);   // this call's end is the next call's reference
        h->have_prev_end = true;
    }
    if (e != RBC_OK) return e;
    return out;
}

size_t footprint(const rbc_ctx *h, int64_t n, int64_t nlip, int64_t nbond) {
    HostSys tmp;
    size_system(h, tmp, n, nlip, nbond);
    return layout(tmp, nullptr);
}

void release(rbc_ctx *h, int32_t slot);

// Everything of an admission but the cell build: validation, allocation, uploads and
// the packed state.  The slot is live and pending.
rbc_status stage(rbc_ctx *h, int32_t slot, int64_t n, const double *x, const double *nrm, const int32_t *type,
                 const double *v, const double *w, int64_t nbond, const int32_t *bonds, const double *r0,
                 const double *box, const int32_t *periodic) {
    if (n < 0 || n > (1ll << 29)) return fail(h, RBC_ERR_INVALID_ARG, "n out of range (at most 2^29 particles)");
    if (n > 0 && (!x || !nrm || !type || !v || !w)) return fail(h, RBC_ERR_INVALID_ARG, "NULL state array");
    if (nbond < 0 || (nbond > 0 && (!bonds || !r0))) return fail(h, RBC_ERR_INVALID_ARG, "bad bond arrays");
    if (!box || !periodic) return fail(h, RBC_ERR_INVALID_ARG, "box and periodic are required");
    double search = h->dprm.cell_search;
    for (int a = 0; a < 3; ++a) {
        if (periodic[a] != 0 && periodic[a] != 1) return fail(h, RBC_ERR_INVALID_ARG, "periodic flags must be 0 or 1");
        if (periodic[a] && !(box[a] > 2.0 * search))
            return fail(h, RBC_ERR_INVALID_ARG, "periodic box length must exceed twice the largest cutoff plus skin");
    }
    if (h->prm.vol_k > 0.0 && (periodic[0] || periodic[1] || periodic[2]))
        return fail(h, RBC_ERR_INVALID_ARG, "the volume constraint needs open boundaries");
    HostSys &hs = h->sys[slot];
    // type histogram and bond topology are needed on the host: wait for the caller's
    // stream, which may still be producing the input arrays
    HIPCHK(hipStreamSynchronize(h->user));
    std::vector<int32_t> ht(n);
    std::vector<int32_t> hb(2 * nbond);
    std::vector<double> hr(nbond);
    if (n > 0) HIPCHK(hipMemcpy(ht.data(), type, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (nbond > 0) {
        HIPCHK(hipMemcpy(hb.data(), bonds, sizeof(int32_t) * 2 * nbond, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(hr.data(), r0, sizeof(double) * nbond, hipMemcpyDeviceToHost));
    }
    std::vector<int32_t> lip;
    for (int64_t i = 0; i < n; ++i) {
        if (ht[i] < 0 || ht[i] > 2) return fail(h, RBC_ERR_INVALID_ARG, "particle type must be 0, 1 or 2");
        if (ht[i] == 0) lip.push_back((int32_t)i);
    }
    const int64_t nlip_real = (int64_t)lip.size();
    if (lip.empty())
        for (int64_t i = 0; i < n; ++i) lip.push_back((int32_t)i);   // no lipids: seed from every particle
    for (int64_t e = 0; e < nbond; ++e)
        if (hb[2 * e] < 0 || hb[2 * e] >= n || hb[2 * e + 1] < 0 || hb[2 * e + 1] >= n || hb[2 * e] == hb[2 * e + 1])
            return fail(h, RBC_ERR_INVALID_ARG, "bond index out of range");
    HostSys fresh;
    size_system(h, fresh, n, nlip_real, nbond);
    if (fresh.nsrcp > 0)                    // the protein set's seeds come from protein beads
        for (int64_t i = 0; i < n; ++i)
            if (ht[i] != 0) lip.push_back((int32_t)i);
    const size_t bytes = layout(fresh, nullptr);
    if (h->budget > 0 && h->used + (int64_t)bytes > h->budget)
        return fail(h, RBC_ERR_CAPACITY, "footprint exceeds the remaining device-memory budget");
    void *mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return fail(h, RBC_ERR_OUT_OF_MEMORY, "device allocation failed");
    if (hipMemset(mem, 0, bytes) != hipSuccess) {
        hipFree(mem);
        return fail(h, RBC_ERR_HIP, "hipMemset of a new system failed");
    }
    // from here on every error path must free the allocation: the slot does not own it yet
    struct FreeOnError {
        void *p;
        ~FreeOnError() {
            if (p) hipFree(p);
        }
    } guard{mem};
    fresh.mem = mem;
    fresh.bytes = bytes;
    layout(fresh, (char *)mem);
    fresh.live = true;
    for (int a = 0; a < 3; ++a) {
        fresh.box[a] = periodic[a] ? box[a] : 0.0;
        fresh.per[a] = periodic[a];
    }
    SysDev &d = fresh.dev;
    d.n = (int32_t)n;
    d.nlip = (int32_t)fresh.nlip;
    d.k = fresh.k;
    d.kl = fresh.kl;
    d.nsrcp = (int32_t)fresh.nsrcp;
    d.nchunk = fresh.nchunk;
    d.split = (n + BLOCK - 1) / BLOCK <= SPLIT_MAX_BLOCKS;
    d.gcap = fresh.gcap;
    d.cnbr_cap = fresh.cnbr_cap;
    d.ntile_p = fresh.ntile_p;
    d.ntile_s = fresh.ntile_s;
    for (int a = 0; a < 3; ++a) { d.per[a] = fresh.per[a]; d.box[a] = fresh.box[a]; }
    // bond CSR by caller id
    std::vector<int32_t> bst(n + 1, 0), bpa(2 * nbond);
    std::vector<double> br(2 * nbond);
    for (int64_t e = 0; e < nbond; ++e) { bst[hb[2 * e] + 1]++; bst[hb[2 * e + 1] + 1]++; }
    for (int64_t i = 0; i < n; ++i) bst[i + 1] += bst[i];
    std::vector<int32_t> fill(n, 0);
    for (int64_t e = 0; e < nbond; ++e) {
        int32_t a = hb[2 * e], b = hb[2 * e + 1];
        int32_t pa = bst[a] + fill[a]++, pb = bst[b] + fill[b]++;
        bpa[pa] = b; br[pa] = hr[e];
        bpa[pb] = a; br[pb] = hr[e];
    }
    HIPCHK(hipMemcpy(d.bstart, bst.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
    if (nbond > 0) {
        HIPCHK(hipMemcpy(d.bpart, bpa.data(), sizeof(int32_t) * 2 * nbond, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d.br0, br.data(), sizeof(double) * 2 * nbond, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(fresh.lip, lip.data(), sizeof(int32_t) * lip.size(), hipMemcpyHostToDevice));
    SysScal zero{};
    HIPCHK(hipMemcpy(h->d_sc + slot, &zero, sizeof(SysScal), hipMemcpyHostToDevice));
    std::memset(h->h_stat + (size_t)slot * STAT_RING, 0, sizeof(StepStat) * STAT_RING);
    hs = fresh;
    guard.p = nullptr;                     // the slot owns the allocation now (release() frees it)
    h->vol_fresh = false;
    h->used += (int64_t)bytes;
    hs.pending = true;
    rbc_status r = refresh_tables(h);
    if (r != RBC_OK) return r;
    {
        Scope sc(h);
        launch_pack(h->L, slot, x, nrm, type, v, w, (int)n);
    }
    HIPCHK(hipStreamSynchronize(h->st));   // the caller may release its input arrays on return
    return RBC_OK;
}

// The initial cell build (seeding and Lloyd iterations, then lists) of the pending
// slots in `which`, in one set of launches.  Slots whose build fails are released
// and listed in `failed`; the first failure's status is returned, with its message.
rbc_status build_pending(rbc_ctx *h, const std::vector<int> &which, std::vector<int> &failed) {
    if (which.empty()) return RBC_OK;
    {
        Scope sc(h);
        run_update(h, which, h->prm.lloyd_iters);
        for (int s : which) {
            HostSys &hs = h->sys[s];
            hs.pending = false;
            hs.steps_since = 0;
            hs.have_stats = false;
            hs.updates = 1;
            hs.rebuilds = 1;
        }
        h->forces_valid = false;
    }
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) return fail(h, RBC_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(le));
    HIPCHK(hipMemcpyAsync(h->h_sc, h->d_sc, sizeof(SysScal) * h->nsys, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    rbc_status first = RBC_OK;
    std::string why;
    for (int s : which) {
        const rbc_status r = slot_error(h, s, h->h_sc[s].err);
        if (r == RBC_OK) continue;
        // the initial cell build failed (capacity, non-finite input): not admitted
        if (first == RBC_OK) {
            first = r;
            why = h->err;
        }
        failed.push_back(s);
    }
    for (int s : failed) {
        release(h, s);
        if (h->d_sc) hipMemset(h->d_sc + s, 0, sizeof(SysScal));
    }
    if (first != RBC_OK) h->err = why;
    return first;
}

rbc_status admit(rbc_ctx *h, int32_t slot, int64_t n, const double *x, const double *nrm, const int32_t *type,
                 const double *v, const double *w, int64_t nbond, const int32_t *bonds, const double *r0,
                 const double *box, const int32_t *periodic) {
    const rbc_status r = stage(h, slot, n, x, nrm, type, v, w, nbond, bonds, r0, box, periodic);
    if (r != RBC_OK) return r;
    std::vector<int> failed;
    return build_pending(h, std::vector<int>{slot}, failed);
}

void release(rbc_ctx *h, int32_t slot) {
    HostSys &hs = h->sys[slot];
    if (!hs.live) return;
    hipStreamSynchronize(h->st);
    if (hs.mem) hipFree(hs.mem);
    if (hs.pairs_mem) hipFree(hs.pairs_mem);
    h->used -= (int64_t)hs.bytes;
    hs = HostSys{};
    refresh_tables(h);
}

rbc_status create(const rbc_params *params, void *stream, int32_t max_slots, int64_t budget, bool ensemble,
                  rbc_handle *out) {
    rbc_ctx *h = nullptr;
    if (!out) return RBC_ERR_INVALID_ARG;
    *out = nullptr;
    std::string why;
    if (!valid_params(params, why)) return RBC_ERR_INVALID_ARG;
    if (max_slots < 1 || max_slots > MAX_SLOTS || budget < 0) return RBC_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return RBC_ERR_HIP;
    h = new rbc_ctx();
    h->prm = *params;
    make_dev_params(h);
    h->max_slots = max_slots;
    h->budget = budget;
    h->ensemble = ensemble;
    h->graphs = false;               // direct launches measured faster; rbc_set_graphs opts in
    h->sys.resize(max_slots);
    h->user = (hipStream_t)stream;
    hipGetDevice(&h->device);
    bool ok = hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&h->ev_out, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&h->d_sys, sizeof(SysDev) * max_slots) == hipSuccess &&
              hipMalloc(&h->d_sc, sizeof(SysScal) * max_slots) == hipSuccess &&
              hipMalloc(&h->d_maps, sizeof(int32_t) * 8 * (max_slots + 1)) == hipSuccess &&
              hipMalloc(&h->d_umaps, sizeof(int32_t) * 7 * (MAX_SLOTS + 1)) == hipSuccess &&
              hipMalloc(&h->d_pmaps, sizeof(int32_t) * (MAX_SLOTS + 1)) == hipSuccess &&
              hipMalloc((void **)&h->d_lip, sizeof(void *) * max_slots) == hipSuccess &&
              hipHostMalloc((void **)&h->h_sc, sizeof(SysScal) * MAX_SLOTS, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&h->h_stat, sizeof(StepStat) * MAX_SLOTS * STAT_RING,
                            hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
              hipHostGetDevicePointer((void **)&h->d_stat, h->h_stat, 0) == hipSuccess;
    if (ok) std::memset(h->h_stat, 0, sizeof(StepStat) * MAX_SLOTS * STAT_RING);
    for (int q = 0; ok && q < RING; ++q) ok = hipEventCreateWithFlags(&h->step_ev[q], hipEventDisableTiming) == hipSuccess;
    if (ok) ok = hipEventCreate(&h->ev_call0) == hipSuccess && hipEventCreate(&h->ev_prev_end) == hipSuccess &&
                 hipEventCreate(&h->ev_prev_end_last) == hipSuccess;
    if (ok) ok = hipMemset(h->d_sc, 0, sizeof(SysScal) * max_slots) == hipSuccess;
    // the allocation-free pair export's staging on this device, looked up once here
    void *ps = nullptr;
    if (ok) ok = pair_scratch_address(h->device, &ps) == hipSuccess;
    h->pair_scratch = (int32_t *)ps;
    if (ok) ok = refresh_tables(h) == RBC_OK;
    if (!ok) {
        rbc_destroy(h);
        return RBC_ERR_HIP;
    }
    *out = h;
    return RBC_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char *rbc_status_string(rbc_status s) {
    switch (s) {
        case RBC_OK: return "ok";
        case RBC_ERR_INVALID_ARG: return "invalid argument";
        case RBC_ERR_OUT_OF_MEMORY: return "out of device memory";
        case RBC_ERR_HIP: return "HIP runtime error";
        case RBC_ERR_NOT_READY: return "no system loaded";
        case RBC_ERR_CAPACITY: return "capacity exceeded";
        case RBC_ERR_NONFINITE: return "non-finite state";
        case RBC_ERR_UNSUPPORTED: return "unsupported parameters";
        case RBC_ERR_SKIN: return "skin exceeded before a cell update";
    }
    return "unknown status";
}

const char *rbc_last_error(rbc_handle h) { return h ? h->err.c_str() : "null handle"; }

rbc_status rbc_create(const rbc_params *params, void *hip_stream, rbc_handle *out) {
    return create(params, hip_stream, 1, 0, false, out);
}

rbc_status rbc_ensemble_create(const rbc_params *params, void *hip_stream, int32_t max_slots, int64_t hbm_budget_bytes,
                               rbc_handle *out) {
    return create(params, hip_stream, max_slots, hbm_budget_bytes, true, out);
}

rbc_status rbc_destroy(rbc_handle h) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (h->st) hipStreamSynchronize(h->st);
    drop_graphs(h);
    for (int s = 0; s < (int)h->sys.size(); ++s) {
        if (h->sys[s].mem) hipFree(h->sys[s].mem);
        if (h->sys[s].pairs_mem) hipFree(h->sys[s].pairs_mem);
    }
    for (auto e : h->tb) hipEventDestroy(e);
    for (auto e : h->te) hipEventDestroy(e);
    for (auto e : h->nb) hipEventDestroy(e);
    for (auto e : h->ne) hipEventDestroy(e);
    for (int q = 0; q < RING; ++q) if (h->step_ev[q]) hipEventDestroy(h->step_ev[q]);
    for (auto e : h->ev_step) hipEventDestroy(e);
    for (hipEvent_t e : {h->ev_call0, h->ev_prev_end, h->ev_prev_end_last})
        if (e) hipEventDestroy(e);
    if (h->d_sys) hipFree(h->d_sys);
    if (h->d_sc) hipFree(h->d_sc);
    if (h->d_maps) hipFree(h->d_maps);
    if (h->d_umaps) hipFree(h->d_umaps);
    if (h->d_pmaps) hipFree(h->d_pmaps);
    if (h->d_lip) hipFree(h->d_lip);
    if (h->h_sc) hipHostFree(h->h_sc);
    if (h->h_stat) hipHostFree(h->h_stat);
    if (h->ev_in) hipEventDestroy(h->ev_in);
    if (h->ev_out) hipEventDestroy(h->ev_out);
    if (h->st) hipStreamDestroy(h->st);
    delete h;
    return RBC_OK;
}

rbc_status rbc_set_system(rbc_handle h, int64_t n, const double *x, const double *nrm, const int32_t *type,
                          const double *v, const double *w, int64_t nbond, const int32_t *bonds, const double *r0,
                          const double *box, const int32_t *periodic) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (h->ensemble) return fail(h, RBC_ERR_INVALID_ARG, "use rbc_ensemble_admit on an ensemble context");
    release(h, 0);
    h->forces_valid = false;
    h->sticky = RBC_OK;
    if (n == 0) return RBC_OK;
    return admit(h, 0, n, x, nrm, type, v, w, nbond, bonds, r0, box, periodic);
}

rbc_status rbc_update_cells(rbc_handle h, int32_t lloyd_iters) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (lloyd_iters < 0) return fail(h, RBC_ERR_INVALID_ARG, "lloyd_iters must be >= 0");
    if (!any_live(h)) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    if (any_pending(h)) return fail(h, RBC_ERR_NOT_READY, "staged systems wait for rbc_ensemble_commit");
    std::vector<int> which;
    for (int s = 0; s < h->nsys; ++s)
        if (runs(h->sys[s])) which.push_back(s);
    {
        Scope sc(h);
        run_update(h, which, lloyd_iters);
        for (int s : which) h->sys[s].have_stats = false;
        h->forces_valid = false;
    }
    return sync_and_check(h);
}

static rbc_status forces_slot(rbc_handle h, int32_t slot, double *F, double *T, double *energy) {
    HostSys &hs = h->sys[slot];
    {
        Scope sc(h);
        force_launch(h, energy != nullptr, 0, 0.0);
        h->forces_valid = true;
        launch_scatter_forces(h->L, slot, F, T, (int)hs.n);
        if (energy) {
            launch_reduce_energy(h->L);
            // U and W are the first two entries of the system's energy record
            hipMemcpyAsync(energy, &h->d_sc[slot].energy[0], 2 * sizeof(double), hipMemcpyDeviceToDevice, h->st);
        }
    }
    return RBC_OK;
}

rbc_status rbc_forces(rbc_handle h, double *F, double *T, double *energy) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (!h->sys[0].live) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    if (any_pending(h)) return fail(h, RBC_ERR_NOT_READY, "staged systems wait for rbc_ensemble_commit");
    return forces_slot(h, 0, F, T, energy);
}

rbc_status rbc_step(rbc_handle h, int64_t nsteps, double dt) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return fail(h, RBC_ERR_INVALID_ARG, "need nsteps >= 0 and dt > 0");
    if (!any_live(h)) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    if (any_pending(h)) return fail(h, RBC_ERR_NOT_READY, "staged systems wait for rbc_ensemble_commit");
    rbc_status r;
    {
        Scope sc(h);
        r = step_all(h, nsteps, dt);
    }
    return r;
}

rbc_status rbc_ensemble_step(rbc_handle h, int64_t nsteps, double dt) { return rbc_step(h, nsteps, dt); }

rbc_status rbc_set_graphs(rbc_handle h, int32_t enable) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (hipStreamSynchronize(h->st) != hipSuccess) return fail(h, RBC_ERR_HIP, "stream synchronisation failed");
    h->graphs = enable != 0;
    if (!h->graphs) drop_graphs(h);
    return RBC_OK;
}

static rbc_status state_slot(rbc_handle h, int32_t slot, double *x, double *nrm, double *v, double *w) {
    if (slot < 0 || slot >= h->max_slots || !h->sys[slot].live) return fail(h, RBC_ERR_NOT_READY, "slot not live");
    if (h->sys[slot].failed != RBC_OK) return fail(h, h->sys[slot].failed, "slot failed: " + h->sys[slot].why);
    Scope sc(h);
    launch_scatter_state(h->L, slot, x, nrm, v, w, (int)h->sys[slot].n);
    return RBC_OK;
}

rbc_status rbc_get_state(rbc_handle h, double *x, double *nrm, double *v, double *w) {
    if (!h) return RBC_ERR_INVALID_ARG;
    return state_slot(h, 0, x, nrm, v, w);
}

rbc_status rbc_ensemble_get_state(rbc_handle h, int32_t slot, double *x, double *nrm, double *v, double *w) {
    if (!h) return RBC_ERR_INVALID_ARG;
    return state_slot(h, slot, x, nrm, v, w);
}

rbc_status rbc_get_pairs(rbc_handle h, int64_t cap, int32_t *ij, int64_t *npairs) {
    if (!h || !npairs || cap < 0 || (cap > 0 && !ij)) return RBC_ERR_INVALID_ARG;
    HostSys &hs = h->sys[0];
    if (!hs.live) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    if (any_pending(h)) return fail(h, RBC_ERR_NOT_READY, "staged systems wait for rbc_ensemble_commit");
    int64_t want = std::max<int64_t>(1024, 32 * hs.n);
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (hs.pairs_cap < want) {
            if (hs.pairs_mem) { hipStreamSynchronize(h->st); hipFree(hs.pairs_mem); }
            hs.pairs_mem = nullptr;
            if (hipMalloc(&hs.pairs_mem, sizeof(int32_t) * 2 * want) != hipSuccess)
                return fail(h, RBC_ERR_OUT_OF_MEMORY, "pair export buffer");
            hs.pairs_cap = want;
            hs.dev.pairs = (int32_t *)hs.pairs_mem;
            hs.dev.pairs_cap = want;
            rbc_status r = refresh_tables(h);
            if (r != RBC_OK) return r;
        }
        int32_t count = 0;
        {
            Scope sc(h);
            HIPCHK(hipMemsetAsync(&h->d_sc[0].npairs, 0, sizeof(int32_t), h->st));
            launch_export_pairs(h->L, 0, (int)hs.n, hs.dev.pairs, hs.pairs_cap, &h->d_sc[0].npairs);
            HIPCHK(hipMemcpyAsync(&count, &h->d_sc[0].npairs, sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
            HIPCHK(hipStreamSynchronize(h->st));
        }
        if (count > hs.pairs_cap) { want = count; continue; }
        std::vector<int32_t> buf(2 * (size_t)count);
        if (count > 0) HIPCHK(hipMemcpy(buf.data(), hs.pairs_mem, sizeof(int32_t) * 2 * count, hipMemcpyDeviceToHost));
        std::vector<int64_t> keys(count);
        for (int32_t q = 0; q < count; ++q) keys[q] = ((int64_t)buf[2 * q] << 32) | (uint32_t)buf[2 * q + 1];
        std::sort(keys.begin(), keys.end());
        const int64_t m = std::min<int64_t>(cap, count);
        for (int64_t q = 0; q < m; ++q) {
            ij[2 * q] = (int32_t)(keys[q] >> 32);
            ij[2 * q + 1] = (int32_t)(keys[q] & 0xffffffff);
        }
        *npairs = count;
        return RBC_OK;
    }
    return fail(h, RBC_ERR_CAPACITY, "pair export overflow");
}

rbc_status rbc_get_pairs_noalloc(rbc_handle h, int64_t cap, int32_t *ij, int64_t *npairs) {
    if (!h || !npairs || cap < 0 || (cap > 0 && !ij)) return RBC_ERR_INVALID_ARG;
    HostSys &hs = h->sys[0];
    if (!hs.live) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    if (any_pending(h)) return fail(h, RBC_ERR_NOT_READY, "staged systems wait for rbc_ensemble_commit");
    if (!h->pair_scratch) return fail(h, RBC_ERR_HIP, "no staging for the allocation-free export on this device");
    int32_t *counter = h->pair_scratch;
    int32_t *out = h->pair_scratch + 64;                 // pairs from byte 256
    int32_t count = 0;
    {
        Scope sc(h);
        launch_zero_counter(h->L, counter);
        launch_export_pairs(h->L, 0, (int)hs.n, out, PAIR_SCRATCH_PAIRS, counter);
        HIPCHK(hipMemcpyAsync(&count, counter, sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
    }
    if ((int64_t)count > PAIR_SCRATCH_PAIRS)
        return fail(h, RBC_ERR_CAPACITY, std::to_string(count) + " pairs exceed the allocation-free export's " +
                                             std::to_string(PAIR_SCRATCH_PAIRS));
    *npairs = count;
    if (cap < count || count == 0) return RBC_OK;        // a size query: nothing written
    HIPCHK(hipMemcpy(ij, out, sizeof(int32_t) * 2 * (size_t)count, hipMemcpyDeviceToHost));
    struct Pair {
        int32_t i, j;
    };
    Pair *p = reinterpret_cast<Pair *>(ij);               // sorted in the caller's buffer, in place
    std::sort(p, p + count, [](const Pair &a, const Pair &b) { return a.i != b.i ? a.i < b.i : a.j < b.j; });
    return RBC_OK;
}

static rbc_status energy_slot(rbc_handle h, int32_t slot, double *out) {
    if (slot < 0 || slot >= h->max_slots || !h->sys[slot].live) return fail(h, RBC_ERR_NOT_READY, "slot not live");
    if (h->sys[slot].failed != RBC_OK) return fail(h, h->sys[slot].failed, "slot failed: " + h->sys[slot].why);
    if (any_pending(h)) return fail(h, RBC_ERR_NOT_READY, "staged systems wait for rbc_ensemble_commit");
    {
        Scope sc(h);
        if (!h->dprm.vol_on) {                        // V is reported with or without the constraint
            launch_volume_partials(h->L);
            launch_volume_reduce(h->L);
        }
        force_launch(h, 1, 0, 0.0);
        h->forces_valid = true;
        launch_reduce_energy(h->L);
    }
    rbc_status r = sync_and_check(h);
    if (r != RBC_OK) return r;
    const double *e = h->h_sc[slot].energy;
    out[0] = e[0];
    out[1] = e[1];
    out[2] = e[2];
    out[3] = e[0] + e[2];
    out[4] = std::sqrt(e[3] * e[3] + e[4] * e[4] + e[5] * e[5]);
    out[5] = std::sqrt(e[6] * e[6] + e[7] * e[7] + e[8] * e[8]);
    out[6] = h->h_sc[slot].volV;
    return RBC_OK;
}

rbc_status rbc_energy(rbc_handle h, double *out) {
    if (!h || !out) return RBC_ERR_INVALID_ARG;
    return energy_slot(h, 0, out);
}

rbc_status rbc_ensemble_energy(rbc_handle h, int32_t slot, double *out) {
    if (!h || !out) return RBC_ERR_INVALID_ARG;
    return energy_slot(h, slot, out);
}

rbc_status rbc_stats(rbc_handle h, int64_t *out) {
    if (!h || !out) return RBC_ERR_INVALID_ARG;
    HostSys &hs = h->sys[0];
    if (!hs.live) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    rbc_status r = sync_and_check(h);
    if (r != RBC_OK) return r;
    out[0] = hs.steps_total;
    out[1] = hs.rebuilds;
    out[2] = hs.early;
    out[3] = hs.k;
    out[4] = h->h_sc[0].nlrows;
    out[5] = h->h_sc[0].cnbr_maxrow;
    out[6] = hs.n;
    out[7] = hs.nlip;
    out[8] = hs.kl;
    out[9] = hs.updates;
    out[10] = hs.prunes;
    return RBC_OK;
}

rbc_status rbc_get_cells(rbc_handle h, int32_t *owner, double *seeds) {
    if (!h) return RBC_ERR_INVALID_ARG;
    HostSys &hs = h->sys[0];
    if (!hs.live) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    if (any_pending(h)) return fail(h, RBC_ERR_NOT_READY, "staged systems wait for rbc_ensemble_commit");
    HIPCHK(hipStreamSynchronize(h->st));
    if (owner) {
        std::vector<int32_t> own(hs.n), gid(hs.n);
        HIPCHK(hipMemcpy(own.data(), hs.dev.owner, sizeof(int32_t) * hs.n, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(gid.data(), hs.dev.gid, sizeof(int32_t) * hs.n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < hs.n; ++i) owner[gid[i]] = own[i];
    }
    if (seeds) {
        std::vector<D4> sd(hs.k);
        HIPCHK(hipMemcpy(sd.data(), hs.dev.seed, sizeof(D4) * hs.k, hipMemcpyDeviceToHost));
        for (int32_t c = 0; c < hs.k; ++c) {
            seeds[3 * c] = sd[c].x;
            seeds[3 * c + 1] = sd[c].y;
            seeds[3 * c + 2] = sd[c].z;
        }
    }
    return RBC_OK;
}

rbc_status rbc_force_timing(rbc_handle h, int32_t enable, double *avg_ms, int64_t *launches) {
    if (!h) return RBC_ERR_INVALID_ARG;
    HIPCHK(hipStreamSynchronize(h->st));
    harvest_timing(h);
    if (avg_ms) *avg_ms = h->tlaunches ? h->tsum_ms / (double)h->tlaunches : 0.0;
    if (launches) *launches = h->tlaunches;
    h->tsum_ms = 0.0;
    h->tlaunches = 0;
    h->timing = enable != 0;
    if (h->timing && h->tb.empty()) {
        h->tb.resize(256);
        h->te.resize(256);
        for (int q = 0; q < 256; ++q) {
            hipEventCreate(&h->tb[q]);
            hipEventCreate(&h->te[q]);
        }
        h->nb.resize(64);
        h->ne.resize(64);
        for (int q = 0; q < 64; ++q) {
            hipEventCreate(&h->nb[q]);
            hipEventCreate(&h->ne[q]);
        }
    }
    return RBC_OK;
}

rbc_status rbc_build_timing(rbc_handle h, double *avg_ms, int64_t *launches) {
    if (!h) return RBC_ERR_INVALID_ARG;
    HIPCHK(hipStreamSynchronize(h->st));
    harvest_timing(h);
    if (avg_ms) *avg_ms = h->nlaunches ? h->nsum_ms / (double)h->nlaunches : 0.0;
    if (launches) *launches = h->nlaunches;
    h->nsum_ms = 0.0;
    h->nlaunches = 0;
    return RBC_OK;
}

rbc_status rbc_debug_array(rbc_handle h, int32_t which, int64_t cap, void *out, int64_t *bytes) {
    if (!h || !bytes || cap < 0 || (cap > 0 && !out)) return RBC_ERR_INVALID_ARG;
    HostSys &hs = h->sys[0];
    if (!hs.live) return fail(h, RBC_ERR_NOT_READY, "no system loaded");
    rbc_status r = sync_and_check(h);
    if (r != RBC_OK && r != RBC_ERR_CAPACITY) return r;
    const SysDev &d = hs.dev;
    const SysScal &sc = h->h_sc[0];
    const void *src = nullptr;
    int64_t nb = 0;
    int32_t total = 0;
    switch (which) {
        case 0: src = d.owner; nb = 4 * hs.n; break;
        case 1: src = d.cstart; nb = 4 * (int64_t)(hs.k + 1); break;
        case 2: src = d.ccount; nb = 4 * (int64_t)hs.k; break;
        case 3: src = d.cnbr_start; nb = 4 * (int64_t)(hs.k + 1); break;
        case 4:
            HIPCHK(hipMemcpy(&total, d.cnbr_start + hs.k, 4, hipMemcpyDeviceToHost));
            src = d.cnbr; nb = 4 * (int64_t)std::min(std::max(total, 0), hs.cnbr_cap); break;
        case 5: src = d.gstart; nb = 4 * (int64_t)(sc.gtot + 1); break;
        case 6: src = d.gseed; nb = 4 * (int64_t)hs.k; break;
        case 7: src = d.seed; nb = sizeof(D4) * (int64_t)hs.k; break;
        case 8: src = d.nlk; nb = 4 * (int64_t)hs.nchunk; break;
        case 9: src = d.scount; nb = 4 * ((hs.n + BLOCK - 1) / BLOCK); break;
        case 10: src = d.gid; nb = 4 * hs.n; break;
        case 11: src = d.tsum; nb = 4 * (int64_t)(std::max((hs.k + SCAN_TILE - 1) / SCAN_TILE, (hs.gcap + SCAN_TILE - 1) / SCAN_TILE) + 2); break;
        case 12: src = d.iscount; nb = 4 * ((hs.n + BLOCK - 1) / BLOCK); break;
        case 13: src = d.ilk; nb = 4 * (int64_t)hs.nchunk; break;
        default: return fail(h, RBC_ERR_INVALID_ARG, "unknown array");
    }
    *bytes = nb;
    if (cap > 0 && nb > 0) HIPCHK(hipMemcpy(out, src, std::min(cap, nb), hipMemcpyDeviceToHost));
    return RBC_OK;
}

rbc_status rbc_sync(rbc_handle h) {
    if (!h) return RBC_ERR_INVALID_ARG;
    return sync_and_check(h);
}

rbc_status rbc_ensemble_footprint(rbc_handle h, int64_t n, int64_t nlip, int64_t nbond, int64_t *bytes) {
    if (!h || !bytes || n <= 0 || nlip < 0 || nlip > n || nbond < 0) return RBC_ERR_INVALID_ARG;
    *bytes = (int64_t)footprint(h, n, nlip, nbond);
    return RBC_OK;
}

rbc_status rbc_ensemble_admit(rbc_handle h, int64_t n, const double *x, const double *nrm, const int32_t *type,
                              const double *v, const double *w, int64_t nbond, const int32_t *bonds, const double *r0,
                              const double *box, const int32_t *periodic, int32_t *slot) {
    if (!h || !slot) return RBC_ERR_INVALID_ARG;
    if (n <= 0) return fail(h, RBC_ERR_INVALID_ARG, "an admitted system needs n > 0");
    int32_t free_slot = -1;
    for (int s = 0; s < h->max_slots; ++s)
        if (!h->sys[s].live) { free_slot = s; break; }
    if (free_slot < 0) return fail(h, RBC_ERR_CAPACITY, "no free slot");
    rbc_status r = admit(h, free_slot, n, x, nrm, type, v, w, nbond, bonds, r0, box, periodic);
    if (r == RBC_OK) *slot = free_slot;
    else release(h, free_slot);
    return r;
}

rbc_status rbc_ensemble_stage(rbc_handle h, int64_t n, const double *x, const double *nrm, const int32_t *type,
                              const double *v, const double *w, int64_t nbond, const int32_t *bonds, const double *r0,
                              const double *box, const int32_t *periodic, int32_t *slot) {
    if (!h || !slot) return RBC_ERR_INVALID_ARG;
    if (n <= 0) return fail(h, RBC_ERR_INVALID_ARG, "an admitted system needs n > 0");
    int32_t free_slot = -1;
    for (int s = 0; s < h->max_slots; ++s)
        if (!h->sys[s].live) { free_slot = s; break; }
    if (free_slot < 0) return fail(h, RBC_ERR_CAPACITY, "no free slot");
    rbc_status r = stage(h, free_slot, n, x, nrm, type, v, w, nbond, bonds, r0, box, periodic);
    if (r == RBC_OK) *slot = free_slot;
    else release(h, free_slot);
    return r;
}

rbc_status rbc_ensemble_commit(rbc_handle h, int64_t cap, int32_t *failed, int64_t *nfailed) {
    if (!h || !nfailed || cap < 0 || (cap > 0 && !failed)) return RBC_ERR_INVALID_ARG;
    std::vector<int> which, bad;
    for (int s = 0; s < h->max_slots; ++s)
        if (h->sys[s].live && h->sys[s].pending) which.push_back(s);
    const rbc_status r = build_pending(h, which, bad);
    *nfailed = (int64_t)bad.size();
    for (size_t q = 0; q < bad.size() && (int64_t)q < cap; ++q) failed[q] = bad[q];
    if (r == RBC_ERR_HIP) return r;
    return RBC_OK;                                // failed builds are reported through the list
}

rbc_status rbc_ensemble_retire(rbc_handle h, int32_t slot) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (slot < 0 || slot >= h->max_slots || !h->sys[slot].live) return fail(h, RBC_ERR_NOT_READY, "slot not live");
    release(h, slot);
    return RBC_OK;
}

rbc_status rbc_ensemble_failed(rbc_handle h, int64_t cap, int32_t *slots, int32_t *status, int64_t *count) {
    if (!h || !count || cap < 0 || (cap > 0 && (!slots || !status))) return RBC_ERR_INVALID_ARG;
    int64_t c = 0;
    for (int s = 0; s < h->max_slots; ++s) {
        const HostSys &hs = h->sys[s];
        if (!hs.live || hs.failed == RBC_OK) continue;
        if (c < cap) {
            slots[c] = s;
            status[c] = (int32_t)hs.failed;
        }
        ++c;
    }
    *count = c;
    return RBC_OK;
}

rbc_status rbc_step_times(rbc_handle h, int32_t enable, int64_t cap, double *ms, int64_t *count, double *gap_ms) {
    if (!h || !count || cap < 0 || (cap > 0 && !ms)) return RBC_ERR_INVALID_ARG;
    const int64_t n = (int64_t)h->step_ms.size();
    for (int64_t q = 0; q < std::min(cap, n); ++q) ms[q] = h->step_ms[q];
    *count = n;
    if (gap_ms) *gap_ms = h->gap_ms;
    const bool on = enable != 0;
    if (on && !h->step_timing) h->have_prev_end = false;   // gaps count from the first timed call
    h->step_timing = on;
    return RBC_OK;
}

rbc_status rbc_host_times(rbc_handle h, double *host_us, double *wait_us) {
    if (!h) return RBC_ERR_INVALID_ARG;
    if (host_us) *host_us = h->host_us_step;
    if (wait_us) *wait_us = h->wait_us_step;
    return RBC_OK;
}

rbc_status rbc_ensemble_info(rbc_handle h, int64_t *out) {
    if (!h || !out) return RBC_ERR_INVALID_ARG;
    int64_t live = 0;
    for (const auto &s : h->sys) live += s.live;
    out[0] = live;
    out[1] = h->used;
    out[2] = h->budget;
    out[3] = h->ens_steps;
    return RBC_OK;
}

}  // extern "C"
