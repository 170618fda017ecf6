// api.hip -- the extern "C" entry points declared in include/swsph.h.
//
// Host side only: argument checks (before any HIP call), workspace layout,
// per-box geometry, and the order of kernel launches for each call.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "launch.h"

using namespace swsph;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return SWSPH_OK;
    return fail(SWSPH_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr uint64_t ALIGN = 256;
uint64_t align_up(uint64_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

struct Geometry {
    int64_t n = 0;
    int32_t n_box = 0;
    int32_t tile = 64;      // most particles per gradient/force tile
    int32_t tile_d = 16;    // most particles per density tile
    int64_t tile_cap = 0;   // most tiles the bin can make (one per particle)
    int64_t n_fine = 0, n_pyr = 0;
    int64_t cand_cap = 0;
    int64_t build_waves = 0;  // most task-build wavefronts (each may hold one list window)
    int tsz = 4;
    std::vector<BoxInfo> boxes;
    Layout lay{};
};

constexpr int KMAX = 10;               // Morton key: 3 x 10 bits per box
constexpr int64_t FINE_MAX = int64_t(1) << 29;

// Candidate-list capacity: 160 entries per particle (lists of cell tiles
// hold ~30-80 per particle on the clustered and uniform sets) plus one
// build window per wavefront that can take one (at most one per tile, at
// most `waves` build wavefronts), below 2^31 (int32 offsets).  Overflow
// latches SWSPH_ST_CAPACITY.
int64_t cand_capacity(int64_t n, int64_t build_waves) {
    const int64_t waves = std::min<int64_t>(std::max<int64_t>(n, 1), build_waves);
    return std::min<int64_t>(160 * n + 65536 + waves * TASK_CHUNK, (int64_t(1) << 31) - 1);
}

// Build wavefronts of a plain plan: BUILD_WAVES_PER_CU per CU.
int64_t default_build_waves() { return (int64_t)device_cu_count() * BUILD_WAVES_PER_CU; }

int choose_k(int64_t nb) {
    // finest grid with about one cell per particle or more (8^k <= 8 nb)
    int k = 0;
    while (k < KMAX && (int64_t(1) << (3 * (k + 1))) <= 8 * nb) ++k;
    return k;
}

int build_geometry(Geometry& G, int64_t n, int32_t n_box, const int64_t* box_count,
                   const double* box_size, int tile, int tile_d, int tsz, int64_t build_waves) {
    if (n < 0) return fail(SWSPH_E_ARG, "n must be >= 0 (got %lld)", (long long)n);
    if (n > (int64_t(1) << 26)) return fail(SWSPH_E_ARG, "n too large (max 2^26)");
    if (n_box < 1) return fail(SWSPH_E_ARG, "n_box must be >= 1");
    if (!box_size) return fail(SWSPH_E_ARG, "box_size (host array) is required");
    if (n_box > 1 && !box_count) return fail(SWSPH_E_ARG, "box_count is required when n_box > 1");
    G.n = n;
    G.n_box = n_box;
    G.tile = tile;
    G.tile_d = tile_d;
    G.tsz = tsz;
    G.boxes.assign(n_box, BoxInfo{});
    int64_t start = 0, fine = 0, pyr = 0, sum = 0;
    for (int b = 0; b < n_box; ++b) {
        const int64_t nb = box_count ? box_count[b] : n;
        const double L = box_size[b];
        if (nb < 0) return fail(SWSPH_E_ARG, "box_count[%d] < 0", b);
        if (!(L > 0) || !std::isfinite(L)) return fail(SWSPH_E_ARG, "box_size[%d] must be > 0", b);
        BoxInfo& bi = G.boxes[b];
        bi.L = L;
        bi.start = start;
        bi.count = nb;
        bi.k = choose_k(nb);
        bi.fine_off = fine;
        bi.pyr_off = pyr;
        start += nb;
        sum += nb;
        fine += int64_t(1) << (3 * bi.k);
        pyr += pyr_level_off(bi.k + 1);
        if (fine > FINE_MAX) return fail(SWSPH_E_ARG, "too many cells (boxes x grid)");
    }
    if (sum != n) return fail(SWSPH_E_ARG, "sum of box_count (%lld) != n (%lld)", (long long)sum,
                              (long long)n);
    G.n_fine = fine;
    G.n_pyr = pyr;
    const int64_t toff = n > 0 ? n : 1;
    G.tile_cap = toff;
    // layout
    Layout& l = G.lay;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + (bytes ? bytes : 1));
        return at;
    };
    const uint64_t N = (uint64_t)n, T = (uint64_t)tsz;
    l.counters = take(sizeof(Counters));
    l.boxtab = take(sizeof(BoxInfo) * n_box);
    l.keys = take(4 * N);
    l.slot = take(4 * N);
    l.tmpidx = take(4 * (N + 1));
    l.perm = take(4 * N);
    l.rank = take(4 * N);
    l.fine_count = take(4 * (uint64_t)(fine + 1));
    l.cstart = take(4 * (uint64_t)(fine + 2));
    l.scan_part = take(4 * (uint64_t)std::max({scan_partials_needed(fine + 1),
                                              scan_partials_needed(n + 1),
                                              scan_partials_needed(order_table_size(n + 1))}));
    l.pos4 = take(4 * T * N);
    l.vel4 = take(4 * T * N);
    l.hs = take(T * N);
    l.dens4 = take(4 * T * N);
    l.hmaxpyr = take(4 * (uint64_t)pyr);
    l.tiles = take(sizeof(Tile) * (uint64_t)toff);
    l.order = take(4 * (uint64_t)toff);
    l.tiles_d = take(sizeof(Tile) * (uint64_t)toff);
    l.order_d = take(4 * (uint64_t)toff);
    l.dparent = take(4 * (uint64_t)(toff + 1));
    l.ord_table = take(4 * (uint64_t)order_table_size(toff));
    l.ord_base = take(4 * (uint64_t)(order_table_size(toff) + 1));
    l.cand_cnt = take(4 * (uint64_t)(toff + 1));
    l.cand_off = take(4 * (uint64_t)(toff + 2));
    G.build_waves = build_waves;
    G.cand_cap = cand_capacity(n, build_waves);
    l.cands = take(4 * (uint64_t)G.cand_cap);
    l.trad = take(4 * (uint64_t)toff);
    l.tflag = take(4 * (uint64_t)toff);
    l.fbox = take(4 * 6 * (uint64_t)toff);
    l.trad_d = take(4 * (uint64_t)toff);
    l.fredo = take(4 * (uint64_t)toff);
    l.forder = take(4 * 2 * (uint64_t)toff);
    // phase words a cache line apart, totals, radii, and the all-boxes word
    l.boxph = take(4 * ((32 + 2) * (uint64_t)n_box + 64));
    l.d_out = take(10 * T * N);
    l.d_int = take(2 * 4 * N);
    l.g_out = take(3 * T * N);
    l.f_out = take(4 * T * N);
    l.f_int = take(4 * N);
    l.adj = take(32 * T * (uint64_t)adj_stride(n));
    l.total = o;
    return SWSPH_OK;
}

}  // namespace

// The bin as the density loop sees it: its own tile set.
BinPtrs swsph::density_view(const BinPtrs& b) {
    BinPtrs d = b;
    d.tiles = b.tiles_d;
    d.order = b.order_d;
    d.ntiles = &b.cnt->n_tiles_d;
    return d;
}

// Pools of HIP event pairs, one list per loop kind.
struct swsph::Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];
    size_t used[4] = {0, 0, 0, 0};
    ~Timer() {
        for (auto& v : ev)
            for (auto& p : v) {
                (void)hipEventDestroy(p.first);
                (void)hipEventDestroy(p.second);
            }
    }
};

void swsph::timer_begin(Timer* t, int loop, hipStream_t s) {
    if (!t) return;
    auto& v = t->ev[loop];
    if (t->used[loop] == v.size()) {
        hipEvent_t a = nullptr, b = nullptr;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
        v.emplace_back(a, b);
    }
    (void)hipEventRecord(v[t->used[loop]].first, s);
}

void swsph::timer_end(Timer* t, int loop, hipStream_t s) {
    if (!t) return;
    auto& v = t->ev[loop];
    if (t->used[loop] >= v.size()) return;
    (void)hipEventRecord(v[t->used[loop]].second, s);
    ++t->used[loop];
}

struct swsph_plan {
    swsph_config cfg;
    swsph::Timer* timer = nullptr;
    int32_t tile, tile_d, lds_cap, lds_cap_d, order, leaf_max;
    bool binned = false;
    void* ws = nullptr;
    Geometry G;
    uint64_t bin_id = 0;
    // captured whole step (swsph_step): its key and the capture stream
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> gkey;
};

namespace {

int check_config(const swsph_config* c) {
    if (!c) return fail(SWSPH_E_ARG, "config is NULL");
    if (!(c->eta > 0) || !(c->eps > 0)) return fail(SWSPH_E_ARG, "eta and eps must be > 0");
    if (!(c->gamma > 1)) return fail(SWSPH_E_ARG, "gamma must be > 1");
    if (!(c->alpha >= 0) || !(c->beta >= 0)) return fail(SWSPH_E_ARG, "alpha, beta must be >= 0");
    if (!(c->h_tol > 0) || !(c->h_tol < 0.1)) return fail(SWSPH_E_ARG, "h_tol must be in (0, 0.1)");
    if (c->h_max_iter < 1 || c->h_max_iter > 1000) return fail(SWSPH_E_ARG, "h_max_iter in [1, 1000]");
    if (c->dtype != SWSPH_F32 && c->dtype != SWSPH_F64) return fail(SWSPH_E_ARG, "bad dtype");
    if (c->tile != 0 && c->tile != 8 && c->tile != 16 && c->tile != 32 && c->tile != 64)
        return fail(SWSPH_E_ARG, "tile must be 0, 8, 16, 32 or 64");
    if (c->tile_dens != 0 && c->tile_dens != 8 && c->tile_dens != 16 && c->tile_dens != 32 &&
        c->tile_dens != 64)
        return fail(SWSPH_E_ARG, "tile_dens must be 0, 8, 16, 32 or 64");
    if (c->lds_cap != 0 && c->lds_cap != 128 && c->lds_cap != 256 && c->lds_cap != 512)
        return fail(SWSPH_E_ARG, "lds_cap must be 0, 128, 256 or 512");
    if (c->lds_cap_dens != 0 && c->lds_cap_dens != 128 && c->lds_cap_dens != 256 &&
        c->lds_cap_dens != 512)
        return fail(SWSPH_E_ARG, "lds_cap_dens must be 0, 128, 256 or 512");
    if (c->order != 0 && c->order != 1) return fail(SWSPH_E_ARG, "order must be 0 or 1");
    if (c->leaf_max < 0 || c->leaf_max > 4096) return fail(SWSPH_E_ARG, "leaf_max in [0, 4096]");
    if ((c->flags & SWSPH_PER_TASK_LAUNCH) && (c->flags & SWSPH_FLAT_LAUNCH))
        return fail(SWSPH_E_ARG, "PER_TASK_LAUNCH and FLAT_LAUNCH are exclusive");
    return SWSPH_OK;
}

int check_particles(const swsph_plan* pl, const swsph_particles* p, bool need_u) {
    if (!p) return fail(SWSPH_E_ARG, "particles is NULL");
    if (p->n < 0) return fail(SWSPH_E_ARG, "n < 0");
    if (p->n > 0) {
        if (!p->x || !p->y || !p->z) return fail(SWSPH_E_ARG, "positions are NULL");
        if (!p->vx || !p->vy || !p->vz) return fail(SWSPH_E_ARG, "velocities are NULL");
        if (!p->m) return fail(SWSPH_E_ARG, "masses are NULL");
        if (need_u && !p->u) return fail(SWSPH_E_ARG, "internal energies are NULL");
    }
    if (p->n_box < 1) return fail(SWSPH_E_ARG, "n_box must be >= 1");
    if (p->n_box > 1 && !p->box_id) return fail(SWSPH_E_ARG, "box_id is required when n_box > 1");
    if (!p->box_size) return fail(SWSPH_E_ARG, "box_size is NULL");
    if ((pl->cfg.flags & SWSPH_FIXED_H) && p->n > 0 && !p->h)
        return fail(SWSPH_E_ARG, "SWSPH_FIXED_H needs particles.h");
    return SWSPH_OK;
}

Scheme scheme_of(const swsph_plan* pl) {
    Scheme s;
    s.eta = pl->cfg.eta;
    s.eps = pl->cfg.eps;
    s.gamma = pl->cfg.gamma;
    s.alpha = pl->cfg.alpha;
    s.beta = pl->cfg.beta;
    s.h_tol = pl->cfg.h_tol;
    s.h_max_iter = pl->cfg.h_max_iter;
    s.flags = pl->cfg.flags;
    s.leaf_max = pl->leaf_max;
    s.order = pl->order;
    s.timer = pl->timer;
    return s;
}

BinPtrs ptrs_of(const swsph_plan* pl, void* ws) {
    const Layout& l = pl->G.lay;
    char* w = (char*)ws;
    BinPtrs b;
    b.cnt = (Counters*)(w + l.counters);
    b.boxtab = (BoxInfo*)(w + l.boxtab);
    b.keys = (uint32_t*)(w + l.keys);
    b.slot = (int32_t*)(w + l.slot);
    b.tmpidx = (int32_t*)(w + l.tmpidx);
    b.perm = (int32_t*)(w + l.perm);
    b.rank = (int32_t*)(w + l.rank);
    b.fine_count = (int32_t*)(w + l.fine_count);
    b.cstart = (int32_t*)(w + l.cstart);
    b.scan_part = (int32_t*)(w + l.scan_part);
    b.pos4 = w + l.pos4;
    b.vel4 = w + l.vel4;
    b.hs = w + l.hs;
    b.dens4 = w + l.dens4;
    b.hmaxpyr = (float*)(w + l.hmaxpyr);
    b.tiles = (Tile*)(w + l.tiles);
    b.order = (int32_t*)(w + l.order);
    b.ntiles = &b.cnt->n_tiles;
    const bool same = pl->G.tile_d == pl->G.tile;
    b.tiles_d = same ? b.tiles : (Tile*)(w + l.tiles_d);
    b.order_d = same ? b.order : (int32_t*)(w + l.order_d);
    b.dparent = (int32_t*)(w + l.dparent);
    b.ord_table = (int32_t*)(w + l.ord_table);
    b.ord_base = (int32_t*)(w + l.ord_base);
    b.cand_cnt = (int32_t*)(w + l.cand_cnt);
    b.cand_off = (int32_t*)(w + l.cand_off);
    b.cands = (uint32_t*)(w + l.cands);
    b.cand_cap = pl->G.cand_cap;
    b.build_waves = pl->G.build_waves;
    b.trad = (float*)(w + l.trad);
    b.tflag = (int32_t*)(w + l.tflag);
    b.fbox = (float*)(w + l.fbox);
    b.trad_d = (float*)(w + l.trad_d);
    b.fredo = (int32_t*)(w + l.fredo);
    b.forder = (int32_t*)(w + l.forder);
    b.boxph = (uint32_t*)(w + l.boxph);
    b.d_out = w + l.d_out;
    b.d_int = (int32_t*)(w + l.d_int);
    b.g_out = w + l.g_out;
    b.f_out = w + l.f_out;
    b.f_int = (int32_t*)(w + l.f_int);
    b.adj = w + l.adj;
    b.n = pl->G.n;
    b.n_box = pl->G.n_box;
    b.tile_cap = pl->G.tile_cap;
    b.tile = pl->G.tile;
    b.tile_d = pl->G.tile_d;
    b.n_fine = pl->G.n_fine;
    b.n_pyr = pl->G.n_pyr;
    return b;
}

int mode_of(const swsph_plan* pl) {
    if (pl->cfg.flags & SWSPH_PER_TASK_LAUNCH) return MODE_PER_TASK;
    if (pl->cfg.flags & SWSPH_FLAT_LAUNCH) return MODE_FLAT;
    return MODE_QUEUE;
}

int check_bound(const swsph_plan* pl, const swsph_particles* p, const void* ws) {
    if (!pl->binned) return fail(SWSPH_E_STATE, "swsph_bin has not been called on this plan");
    if (ws != pl->ws) return fail(SWSPH_E_STATE, "workspace differs from the one passed to swsph_bin");
    if (p->n != pl->G.n || p->n_box != pl->G.n_box)
        return fail(SWSPH_E_STATE, "particle count / boxes differ from the last swsph_bin");
    return SWSPH_OK;
}

template <typename T>
void unsort_density(const BinPtrs& b, swsph_density_out* o, hipStream_t s) {
    const int64_t n = b.n;
    T* d = (T*)b.d_out;
    void* dst[10] = {o->h, o->rho, o->rho_dh, o->wcount, o->wcount_dh,
                     o->div_v, o->curl_x, o->curl_y, o->curl_z, o->f};
    UnsortSet u{};
    for (int k = 0; k < 10; ++k) {
        u.in[k] = d + k * n;
        u.out[k] = dst[k];
    }
    u.k = 10;
    launch_unsort_multi<T>(n, b.rank, u, s);
    UnsortSet ui{};
    ui.in[0] = b.d_int;
    ui.out[0] = o->nngb;
    ui.in[1] = b.d_int + n;
    ui.out[1] = o->iters;
    ui.k = 2;
    if (o->nngb || o->iters) launch_unsort_multi<int32_t>(n, b.rank, ui, s);
}

}  // namespace

extern "C" {

int swsph_version(void) { return SWSPH_VERSION; }

const char* swsph_last_error(void) { return g_err.c_str(); }

void swsph_config_default(swsph_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof *c);
    c->eta = 1.2348;
    c->eps = 2.0;
    c->gamma = 5.0 / 3.0;
    c->alpha = 1.0;
    c->beta = 3.0;
    c->h_tol = 2e-6;
    c->h_max_iter = 40;
    c->dtype = SWSPH_F32;
    c->flags = 0;
    c->tile = 0;
    c->lds_cap = 0;
    c->order = 1;
    c->leaf_max = 0;
}

int swsph_plan_create(swsph_plan** out, const swsph_config* cfg) {
    if (!out) return fail(SWSPH_E_ARG, "out is NULL");
    *out = nullptr;
    int r = check_config(cfg);
    if (r) return r;
    swsph_plan* pl = new (std::nothrow) swsph_plan();
    if (!pl) return fail(SWSPH_E_ARG, "out of host memory");
    pl->cfg = *cfg;
    pl->tile = cfg->tile ? cfg->tile : 64;
    pl->tile_d = cfg->tile_dens ? cfg->tile_dens : 16;
    pl->lds_cap = cfg->lds_cap ? cfg->lds_cap : 128;
    pl->lds_cap_d = cfg->lds_cap_dens ? cfg->lds_cap_dens : 512;
    pl->order = cfg->order;
    pl->leaf_max = cfg->leaf_max ? cfg->leaf_max : 64;
    if (cfg->flags & SWSPH_TIMING) pl->timer = new (std::nothrow) swsph::Timer();
    *out = pl;
    return SWSPH_OK;
}

int swsph_plan_destroy(swsph_plan* pl) {
    if (pl) {
        delete pl->timer;
        if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
        if (pl->cap) (void)hipStreamDestroy(pl->cap);
    }
    delete pl;
    return SWSPH_OK;
}

int swsph_plan_get_tuning(const swsph_plan* pl, swsph_tuning* out) {
    if (!pl || !out) return fail(SWSPH_E_ARG, "plan and out are required");
    out->tile = pl->tile;
    out->tile_dens = pl->tile_d;
    out->lds_cap = pl->lds_cap;
    out->lds_cap_dens = pl->lds_cap_d;
    out->order = pl->order;
    out->leaf_max = pl->leaf_max;
    return SWSPH_OK;
}

int swsph_workspace_bytes(const swsph_plan* pl, int64_t n, int32_t n_box, const int64_t* box_count,
                          const double* box_size, uint64_t* bytes) {
    if (!pl || !bytes) return fail(SWSPH_E_ARG, "plan and bytes are required");
    Geometry G;
    int r = build_geometry(G, n, n_box, box_count, box_size, pl->tile, pl->tile_d,
                           pl->cfg.dtype == SWSPH_F64 ? 8 : 4, default_build_waves());
    if (r) return r;
    *bytes = G.lay.total;
    return SWSPH_OK;
}

}  // extern "C"

namespace {

// swsph_bin in three parts: host checks and geometry (plan state), the box
// table upload, and the binning kernels (capturable: no host memory).
int bin_prepare(swsph_plan* pl, const swsph_particles* p, void* ws,
                int64_t build_waves = default_build_waves()) {
    int r = check_particles(pl, p, false);
    if (r) return r;
    if (!ws) return fail(SWSPH_E_ARG, "workspace is NULL");
    if (((uintptr_t)ws) % ALIGN) return fail(SWSPH_E_ARG, "workspace must be 256-byte aligned");
    Geometry G;
    const int64_t one = p->n;
    r = build_geometry(G, p->n, p->n_box, p->box_count ? p->box_count : &one, p->box_size,
                       pl->tile, pl->tile_d, pl->cfg.dtype == SWSPH_F64 ? 8 : 4, build_waves);
    if (r) return r;
    pl->G = G;
    pl->ws = ws;
    pl->binned = true;
    ++pl->bin_id;
    return SWSPH_OK;
}

int bin_upload(swsph_plan* pl, hipStream_t s) {
    BinPtrs b = ptrs_of(pl, pl->ws);
    return hip_check(hipMemcpyAsync(b.boxtab, pl->G.boxes.data(), sizeof(BoxInfo) * pl->G.n_box,
                                    hipMemcpyHostToDevice, s),
                     "copy box table");
}

void bin_enqueue(swsph_plan* pl, const swsph_particles* p, hipStream_t s) {
    const Geometry& G = pl->G;
    BinPtrs b = ptrs_of(pl, pl->ws);
    launch_fill_u32(b.cnt, sizeof(Counters) / 4, 0u, s);
    launch_fill_u32(b.fine_count, G.n_fine + 1, 0u, s);
    const bool f64 = pl->cfg.dtype == SWSPH_F64;
    if (f64) launch_keys<double>(p, b.boxtab, b.keys, b.slot, b.fine_count, b.cnt, s);
    else launch_keys<float>(p, b.boxtab, b.keys, b.slot, b.fine_count, b.cnt, s);
    launch_exclusive_scan(b.fine_count, G.n_fine, b.scan_part, b.cstart, s);
    launch_box_check(G.n_box, b.boxtab, b.cstart, b.cnt, s);
    launch_scatter_stable(G.n, b.keys, b.slot, b.cstart, b.tmpidx, b.perm, b.rank, b.cnt, s);
    if (f64) {
        launch_gather<double>(p, b.boxtab, b.keys, b.cstart, b.perm, pl->cfg.eta, b.pos4, b.vel4,
                              b.hs, s);
        launch_make_tiles<double>(b, s);
    } else {
        launch_gather<float>(p, b.boxtab, b.keys, b.cstart, b.perm, pl->cfg.eta, b.pos4, b.vel4,
                             b.hs, s);
        launch_make_tiles<float>(b, s);
    }
}

}  // namespace

extern "C" {

int swsph_bin(swsph_plan* pl, const swsph_particles* p, void* ws, void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    int r = bin_prepare(pl, p, ws);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    r = bin_upload(pl, s);
    if (r) return r;
    bin_enqueue(pl, p, s);
    return hip_check(hipGetLastError(), "swsph_bin launch");
}

int swsph_density(swsph_plan* pl, const swsph_particles* p, swsph_density_out* o, void* ws,
                  void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    int r = check_particles(pl, p, false);
    if (r) return r;
    if (!o || (p->n > 0 && (!o->h || !o->rho || !o->f)))
        return fail(SWSPH_E_ARG, "density output needs h, rho and f");
    r = check_bound(pl, p, ws);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    BinPtrs b = ptrs_of(pl, ws);
    Scheme sc = scheme_of(pl);
    const int mode = mode_of(pl);
    if (pl->cfg.dtype == SWSPH_F64) {
        r = launch_density<double>(b, sc, mode, pl->lds_cap_d, s);
        unsort_density<double>(b, o, s);
    } else {
        r = launch_density<float>(b, sc, mode, pl->lds_cap_d, s);
        unsort_density<float>(b, o, s);
    }
    if (r) return fail(SWSPH_E_HIP, "density kernel launch failed");
    return hip_check(hipGetLastError(), "density");
}

}  // extern "C"

namespace {

// Gradient and/or force over one density result: the density fields are
// gathered into binned order, the task lists built, and one loop kernel
// computes both loops (the outputs asked for are copied out), so the
// separate calls and the joint one give the same bits.
// The binned gradient and force results back to the caller's order.
template <typename T>
void gf_unsort(const BinPtrs& b, swsph_gradient_out* go, swsph_force_out* fo, hipStream_t s) {
    const int64_t n = b.n;
    UnsortSet u{};
    if (go) {
        u.in[u.k] = (T*)b.g_out;
        u.out[u.k++] = go->v_sig;
        u.in[u.k] = (T*)b.g_out + n;
        u.out[u.k++] = go->lap_u;
    }
    if (fo) {
        void* dst[4] = {fo->ax, fo->ay, fo->az, fo->dudt};
        for (int k = 0; k < 4; ++k) {
            u.in[u.k] = (T*)b.f_out + k * n;
            u.out[u.k++] = dst[k];
        }
        if (fo->nint) launch_unsort<int32_t>(n, b.rank, b.f_int, fo->nint, s);
    }
    launch_unsort_multi<T>(n, b.rank, u, s);
}

template <typename T>
int gf_enqueue(swsph_plan* pl, const swsph_particles* p, const swsph_density_out* d,
               swsph_gradient_out* go, swsph_force_out* fo, void* ws, hipStream_t s) {
    BinPtrs b = ptrs_of(pl, ws);
    Scheme sc = scheme_of(pl);
    const int mode = mode_of(pl);
    (void)p;
    launch_prep_dens<T>(b, sc, d, s);
    launch_gf_tasks<T>(b, sc, s);
    if (launch_force<T>(b, sc, mode, pl->lds_cap, s))
        return fail(SWSPH_E_HIP, "gradient/force kernel launch failed");
    gf_unsort<T>(b, go, fo, s);
    return hip_check(hipGetLastError(), go ? (fo ? "gradient+force" : "gradient") : "force");
}

// The single-launch step after the bin: density, gradient and force loops
// of every box in one launch (and the separate-launch path for what it
// leaves), then the results in the caller's order.
template <typename T>
int single_enqueue(swsph_plan* pl, swsph_density_out* d, swsph_gradient_out* go,
                   swsph_force_out* fo, void* ws, hipStream_t s) {
    BinPtrs b = ptrs_of(pl, ws);
    Scheme sc = scheme_of(pl);
    if (launch_single<T>(b, sc, pl->lds_cap_d, pl->lds_cap, s))
        return fail(SWSPH_E_HIP, "single-launch loop kernel launch failed");
    unsort_density<T>(b, d, s);
    gf_unsort<T>(b, go, fo, s);
    return hip_check(hipGetLastError(), "single-launch step");
}

// Whether swsph_step takes the single launch: asked for, both gradient/force
// outputs wanted, and density tiles smaller than gradient/force tiles (they
// stage from their gradient/force tile's list).
bool single_launch(const swsph_plan* pl, const swsph_gradient_out* go, const swsph_force_out* fo) {
    return (pl->cfg.flags & SWSPH_SINGLE_LAUNCH) && !(pl->cfg.flags & SWSPH_PER_TASK_LAUNCH) &&
           (go || fo) && pl->tile_d < pl->tile;
}

int single_checked(swsph_plan* pl, const swsph_particles* p, swsph_density_out* d,
                   swsph_gradient_out* go, swsph_force_out* fo, void* ws, void* stream) {
    int r = check_particles(pl, p, true);
    if (r) return r;
    if (!d || (p->n > 0 && (!d->h || !d->rho || !d->f)))
        return fail(SWSPH_E_ARG, "density output needs h, rho and f");
    r = check_bound(pl, p, ws);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    return pl->cfg.dtype == SWSPH_F64 ? single_enqueue<double>(pl, d, go, fo, ws, s)
                                      : single_enqueue<float>(pl, d, go, fo, ws, s);
}

int gf_checked(swsph_plan* pl, const swsph_particles* p, const swsph_density_out* d,
               swsph_gradient_out* go, swsph_force_out* fo, void* ws, void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    int r = check_particles(pl, p, true);
    if (r) return r;
    if (!d || (p->n > 0 && (!d->h || !d->rho || !d->f)))
        return fail(SWSPH_E_ARG, "gradient and force need density h, rho and f");
    r = check_bound(pl, p, ws);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    return pl->cfg.dtype == SWSPH_F64 ? gf_enqueue<double>(pl, p, d, go, fo, ws, s)
                                      : gf_enqueue<float>(pl, p, d, go, fo, ws, s);
}

}  // namespace

extern "C" {

int swsph_gradient(swsph_plan* pl, const swsph_particles* p, const swsph_density_out* d,
                   swsph_gradient_out* o, void* ws, void* stream) {
    if (pl && !o) return fail(SWSPH_E_ARG, "gradient output is NULL");
    return gf_checked(pl, p, d, o, nullptr, ws, stream);
}

int swsph_force(swsph_plan* pl, const swsph_particles* p, const swsph_density_out* d,
                swsph_force_out* o, void* ws, void* stream) {
    if (pl && !o) return fail(SWSPH_E_ARG, "force output is NULL");
    return gf_checked(pl, p, d, nullptr, o, ws, stream);
}

int swsph_gradient_force(swsph_plan* pl, const swsph_particles* p, const swsph_density_out* d,
                         swsph_gradient_out* go, swsph_force_out* fo, void* ws, void* stream) {
    if (pl && (!go || !fo)) return fail(SWSPH_E_ARG, "gradient and force outputs are required");
    return gf_checked(pl, p, d, go, fo, ws, stream);
}

int swsph_gradient_force_sw(swsph_plan* pl, const swsph_particles* p, const swsph_density_out* d,
                            const swsph_switch_params* sp, swsph_switch_state* st,
                            swsph_gradient_out* go, swsph_force_out* fo, void* ws,
                            void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    int r = check_particles(pl, p, true);
    if (r) return r;
    if (!d || (p->n > 0 && (!d->h || !d->rho || !d->f || !d->div_v || !d->curl_x ||
                            !d->curl_y || !d->curl_z)))
        return fail(SWSPH_E_ARG, "switches need density h, rho, f, div_v and curl_x/y/z");
    if (!sp) return fail(SWSPH_E_ARG, "switch parameters are NULL");
    if (!(sp->dt > 0) || !(sp->av_max > 0) || !(sp->av_min >= 0) || !(sp->ell >= 0) ||
        !(sp->beta_c >= 0) || !(sp->ac_min >= 0) || !(sp->ac_max >= sp->ac_min) ||
        !(sp->bal_eps >= 0))
        return fail(SWSPH_E_ARG, "switch parameters out of range (dt > 0, av_max > 0, "
                                 "av_min, ell, beta_c, ac_min, bal_eps >= 0, ac_max >= ac_min)");
    if (!st || (p->n > 0 && (!st->alpha_v || !st->alpha_c || !st->div_v_prev || !st->v_sig_prev)))
        return fail(SWSPH_E_ARG, "switch state needs alpha_v, alpha_c, div_v_prev, v_sig_prev");
    if (!go || !fo || (p->n > 0 && (!go->v_sig || !go->lap_u || !fo->ax || !fo->ay || !fo->az ||
                                     !fo->dudt)))
        return fail(SWSPH_E_ARG, "gradient and force outputs are required");
    r = check_bound(pl, p, ws);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    BinPtrs b = ptrs_of(pl, ws);
    Scheme sc = scheme_of(pl);
    const int mode = mode_of(pl);
    const int64_t n = b.n;
    const SwitchConsts sw{sp->dt, sp->av_max, sp->av_min, sp->ell, sp->beta_c, sp->ac_min,
                          sp->ac_max, sp->bal_eps};
    const bool f64 = pl->cfg.dtype == SWSPH_F64;
    if (f64) {
        launch_prep_dens<double>(b, sc, d, s);
        launch_gf_tasks<double>(b, sc, s);
        r = launch_switch_loops<double>(b, sc, sw, d, st, mode, pl->lds_cap, s);
    } else {
        launch_prep_dens<float>(b, sc, d, s);
        launch_gf_tasks<float>(b, sc, s);
        r = launch_switch_loops<float>(b, sc, sw, d, st, mode, pl->lds_cap, s);
    }
    if (r) return fail(SWSPH_E_HIP, "switch loop launch failed");
    const size_t tsz = f64 ? 8 : 4;
    UnsortSet u{};
    u.in[0] = b.g_out;
    u.out[0] = go->v_sig;
    u.in[1] = (char*)b.g_out + tsz * n;
    u.out[1] = go->lap_u;
    void* dst[4] = {fo->ax, fo->ay, fo->az, fo->dudt};
    for (int k = 0; k < 4; ++k) {
        u.in[2 + k] = (char*)b.f_out + tsz * k * n;
        u.out[2 + k] = dst[k];
    }
    u.k = 6;
    if (f64) launch_unsort_multi<double>(n, b.rank, u, s);
    else launch_unsort_multi<float>(n, b.rank, u, s);
    if (fo->nint) launch_unsort<int32_t>(n, b.rank, b.f_int, fo->nint, s);
    return hip_check(hipGetLastError(), "gradient+force with switches");
}

int swsph_kick_drift(const swsph_plan* pl, int64_t n, void* x, void* y, void* z, void* vx,
                     void* vy, void* vz, void* u, const void* ax, const void* ay,
                     const void* az, const void* dudt, double dt_kick, double dt_drift,
                     const int32_t* box_id, int32_t n_box, const double* box_size,
                     void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    if (n < 0) return fail(SWSPH_E_ARG, "n < 0");
    if (!std::isfinite(dt_kick) || !std::isfinite(dt_drift))
        return fail(SWSPH_E_ARG, "time steps must be finite");
    if (n_box < 1 || n_box > DRIFT_MAX_BOXES)
        return fail(SWSPH_E_ARG, "n_box must be in [1, %d]", DRIFT_MAX_BOXES);
    if (n_box > 1 && !box_id) return fail(SWSPH_E_ARG, "box_id is required when n_box > 1");
    if (!box_size) return fail(SWSPH_E_ARG, "box_size is NULL");
    DriftBoxes boxes{};
    for (int b = 0; b < n_box; ++b) {
        if (!(box_size[b] > 0) || !std::isfinite(box_size[b]))
            return fail(SWSPH_E_ARG, "box_size[%d] must be > 0", b);
        boxes.L[b] = box_size[b];
    }
    if (n > 0) {
        if (!vx || !vy || !vz) return fail(SWSPH_E_ARG, "velocities are NULL");
        if (dt_kick != 0.0 && (!u || !ax || !ay || !az || !dudt))
            return fail(SWSPH_E_ARG, "a kick needs u, a and du/dt");
        if (dt_drift != 0.0 && (!x || !y || !z)) return fail(SWSPH_E_ARG, "positions are NULL");
    }
    hipStream_t s = (hipStream_t)stream;
    if (pl->cfg.dtype == SWSPH_F64)
        launch_kick_drift<double>(n, x, y, z, vx, vy, vz, u, ax, ay, az, dudt, dt_kick, dt_drift,
                                  box_id, n_box, boxes, s);
    else
        launch_kick_drift<float>(n, x, y, z, vx, vy, vz, u, ax, ay, az, dudt, dt_kick, dt_drift,
                                 box_id, n_box, boxes, s);
    return hip_check(hipGetLastError(), "kick/drift");
}

int swsph_kernel_times(swsph_plan* pl, double ms[4], uint64_t launches[4], void* stream) {
    if (!pl || !ms || !launches) return fail(SWSPH_E_ARG, "plan, ms and launches are required");
    for (int k = 0; k < 4; ++k) { ms[k] = 0.0; launches[k] = 0; }
    if (!pl->timer) return SWSPH_OK;
    int r = hip_check(hipStreamSynchronize((hipStream_t)stream), "synchronise");
    if (r) return r;
    for (int k = 0; k < 4; ++k) {
        double tot = 0.0;
        for (size_t i = 0; i < pl->timer->used[k]; ++i) {
            float e = 0.f;
            if (hipEventElapsedTime(&e, pl->timer->ev[k][i].first, pl->timer->ev[k][i].second) ==
                hipSuccess)
                tot += e;
        }
        launches[k] = pl->timer->used[k];
        ms[k] = launches[k] ? tot / (double)launches[k] : 0.0;
    }
    return SWSPH_OK;
}

int swsph_reset_timers(swsph_plan* pl) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    if (pl->timer)
        for (int k = 0; k < 4; ++k) pl->timer->used[k] = 0;
    return SWSPH_OK;
}

int swsph_read_stats(swsph_plan* pl, const void* ws, swsph_stats* out, void* stream) {
    if (!pl || !out) return fail(SWSPH_E_ARG, "plan and out are required");
    if (!ws) ws = pl->ws;  // the workspace of the plan's last bin (swsph_step_static's scratch)
    if (!ws) return fail(SWSPH_E_STATE, "no bin on this plan");
    if (!pl->binned || ws != pl->ws) return fail(SWSPH_E_STATE, "no bin on this workspace");
    Counters c;
    hipStream_t s = (hipStream_t)stream;
    int r = hip_check(hipMemcpyAsync(&c, (const char*)ws + pl->G.lay.counters, sizeof c,
                                     hipMemcpyDeviceToHost, s),
                      "read stats");
    if (r) return r;
    r = hip_check(hipStreamSynchronize(s), "synchronise");
    if (r) return r;
    std::memset(out, 0, sizeof *out);
    out->status = (uint32_t)c.status;
    out->n_tiles = (uint32_t)c.n_tiles;
    for (int k = 0; k < 4; ++k) {
        out->pairs_tested[k] = c.pairs_tested[k];
        out->pairs_inside[k] = c.pairs_inside[k];
    }
    out->newton_sweeps = c.newton_sweeps;
    out->newton_max = (uint32_t)c.newton_max;
    out->newton_failed = (uint32_t)c.newton_failed;
    out->listed = c.listed;
    out->restages = c.restages;
    out->n_tiles_dens = c.n_tiles_d;
    out->dens_listed = c.dens_listed;
    out->single_redo = c.single_redo;
    if (c.status & SWSPH_ST_DOMAIN) return fail(SWSPH_E_DOMAIN, "a particle lies outside its box");
    if (c.status & SWSPH_ST_REACH) return fail(SWSPH_E_REACH, "a support radius reaches half a box");
    if (c.status & SWSPH_ST_CAPACITY) return fail(SWSPH_E_CAPACITY, "internal capacity exceeded");
    if (c.status & SWSPH_ST_LOOPCAP) return fail(SWSPH_E_CAPACITY, "a device loop hit its cap");
    if (c.status & SWSPH_ST_NEWTON) return fail(SWSPH_E_NEWTON, "Newton iteration did not converge");
    return SWSPH_OK;
}

}  // extern "C"

namespace {

// Everything a captured step depends on: pointers, sizes, box data and the
// execution options.  A different key means a new capture.
std::vector<uint64_t> step_key(const swsph_plan* pl, const swsph_particles* p,
                               const swsph_density_out* d, const swsph_gradient_out* go,
                               const swsph_force_out* fo, const void* ws) {
    std::vector<uint64_t> k;
    auto P = [&](const void* v) { k.push_back((uint64_t)(uintptr_t)v); };
    P(ws);
    k.push_back((uint64_t)p->n);
    k.push_back((uint64_t)p->n_box);
    P(p->x); P(p->y); P(p->z); P(p->vx); P(p->vy); P(p->vz); P(p->u); P(p->m);
    P(p->box_id); P(p->h);
    for (int b = 0; b < p->n_box; ++b) {
        uint64_t bits;
        std::memcpy(&bits, &p->box_size[b], 8);
        k.push_back(bits);
        k.push_back(p->box_count ? (uint64_t)p->box_count[b] : (uint64_t)p->n);
    }
    P(d->h); P(d->rho); P(d->rho_dh); P(d->wcount); P(d->wcount_dh); P(d->div_v);
    P(d->curl_x); P(d->curl_y); P(d->curl_z); P(d->f); P(d->nngb); P(d->iters);
    P(go); if (go) { P(go->v_sig); P(go->lap_u); }
    P(fo); if (fo) { P(fo->ax); P(fo->ay); P(fo->az); P(fo->dudt); P(fo->nint); }
    const swsph_config& c = pl->cfg;
    const double dv[6] = {c.eta, c.eps, c.gamma, c.alpha, c.beta, c.h_tol};
    for (double v : dv) {
        uint64_t bits;
        std::memcpy(&bits, &v, 8);
        k.push_back(bits);
    }
    k.push_back((uint64_t)c.h_max_iter);
    k.push_back((uint64_t)c.dtype);
    k.push_back((uint64_t)c.flags);
    k.push_back((uint64_t)pl->tile);
    k.push_back((uint64_t)pl->tile_d);
    k.push_back((uint64_t)pl->lds_cap);
    k.push_back((uint64_t)pl->lds_cap_d);
    k.push_back((uint64_t)pl->order);
    k.push_back((uint64_t)pl->leaf_max);
    return k;
}

int step_eager(swsph_plan* pl, const swsph_particles* p, swsph_density_out* d,
               swsph_gradient_out* go, swsph_force_out* fo, void* ws, void* stream) {
    int r = swsph_bin(pl, p, ws, stream);
    if (r) return r;
    if (single_launch(pl, go, fo)) return single_checked(pl, p, d, go, fo, ws, stream);
    r = swsph_density(pl, p, d, ws, stream);
    if (r) return r;
    if (go || fo) return gf_checked(pl, p, d, go, fo, ws, stream);
    return SWSPH_OK;
}

void drop_graph(swsph_plan* pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    pl->exec = nullptr;
    pl->gkey.clear();
}

}  // namespace

extern "C" {

int swsph_step(swsph_plan* pl, const swsph_particles* p, swsph_density_out* d,
               swsph_gradient_out* go, swsph_force_out* fo, void* ws, void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    if (!d) return fail(SWSPH_E_ARG, "density output is NULL");
    int r = check_particles(pl, p, true);
    if (r) return r;
    // one launch per task reads the task count back, and timing records
    // events: both run eagerly
    if (pl->cfg.flags & (SWSPH_PER_TASK_LAUNCH | SWSPH_TIMING) || p->n == 0)
        return step_eager(pl, p, d, go, fo, ws, stream);
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint64_t> key = step_key(pl, p, d, go, fo, ws);
    if (!pl->exec || key != pl->gkey) {
        drop_graph(pl);
        r = bin_prepare(pl, p, ws);
        if (r) return r;
        r = bin_upload(pl, s);
        if (r) return r;
        if (!pl->cap) {
            r = hip_check(hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking), "capture stream");
            if (r) return r;
        }
        r = hip_check(hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal), "begin capture");
        if (r) return r;
        bin_enqueue(pl, p, pl->cap);
        int rr = 0;
        if (single_launch(pl, go, fo)) {
            rr = single_checked(pl, p, d, go, fo, ws, pl->cap);
        } else {
            rr = swsph_density(pl, p, d, ws, pl->cap);
            if (!rr && (go || fo)) rr = gf_checked(pl, p, d, go, fo, ws, pl->cap);
        }
        hipGraph_t g = nullptr;
        r = hip_check(hipStreamEndCapture(pl->cap, &g), "end capture");
        if (!r && rr) r = rr;
        if (!r) r = hip_check(hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0), "instantiate");
        if (g) (void)hipGraphDestroy(g);
        if (r) {
            drop_graph(pl);
            return r;
        }
        pl->gkey = std::move(key);
    } else {
        // Another bin on this plan (an eager call, or swsph_bin of other
        // particles) may have rewritten the plan's geometry and the box
        // table in the workspace since the capture: restore both for the
        // captured particles before the replay reads them.
        r = bin_prepare(pl, p, ws);
        if (r) return r;
        r = bin_upload(pl, s);
        if (r) return r;
    }
    return hip_check(hipGraphLaunch(pl->exec, s), "graph launch");
}

}  // extern "C"

namespace {

// Library-owned scratch of swsph_step_static: a file-scope device array, one
// copy on every GPU the library runs on, held until the process ends.  Host
// code never uses the array's name as an address: the device address of
// each GPU's copy comes from hipGetSymbolAddress, once per device.
constexpr uint64_t STATIC_SCRATCH_BYTES = SWSPH_STATIC_SCRATCH_BYTES;
// Task-build wavefronts of a static step: each may hold one candidate-list
// window of TASK_CHUNK entries, so fewer of them leave the scratch to the
// particles (the builds of small sets do not fill more).
constexpr int64_t STATIC_BUILD_WAVES = 256;
__device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current GPU's scratch (looked up on first use).
int static_scratch(void** out) {
    int dev = 0;
    int r = hip_check(hipGetDevice(&dev), "get device");
    if (r) return r;
    if (dev < 0 || dev >= MAX_DEVICES) return fail(SWSPH_E_ARG, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        r = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (r) return r;
        if (!ptr || ((uintptr_t)ptr) % ALIGN) return fail(SWSPH_E_HIP, "scratch address unusable");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SWSPH_OK;
}

}  // namespace

extern "C" {

int swsph_step_static(swsph_plan* pl, const swsph_particles* p, swsph_density_out* d,
                      swsph_gradient_out* go, swsph_force_out* fo, void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    if (!d) return fail(SWSPH_E_ARG, "density output is NULL");
    int r = check_particles(pl, p, true);
    if (r) return r;
    // size check before anything else (plan state and device untouched)
    Geometry G;
    const int64_t one = p->n;
    r = build_geometry(G, p->n, p->n_box, p->box_count ? p->box_count : &one, p->box_size,
                       pl->tile, pl->tile_d, pl->cfg.dtype == SWSPH_F64 ? 8 : 4,
                       STATIC_BUILD_WAVES);
    if (r) return r;
    if (G.lay.total > STATIC_SCRATCH_BYTES)
        return fail(SWSPH_E_ARG,
                    "swsph_step_static: %lld particles need %llu bytes of scratch, more than the "
                    "%llu bytes of the static scratch (use swsph_step with a workspace)",
                    (long long)p->n, (unsigned long long)G.lay.total,
                    (unsigned long long)STATIC_SCRATCH_BYTES);
    void* ws = nullptr;
    r = static_scratch(&ws);
    if (r) return r;
    r = bin_prepare(pl, p, ws, STATIC_BUILD_WAVES);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    r = bin_upload(pl, s);
    if (r) return r;
    // the bin clears the counters, queue heads and histograms the kernels
    // count from, so whatever a previous call left in the scratch is unused
    bin_enqueue(pl, p, s);
    r = hip_check(hipGetLastError(), "swsph_step_static bin");
    if (r) return r;
    r = swsph_density(pl, p, d, ws, stream);
    if (r) return r;
    if (go || fo) return gf_checked(pl, p, d, go, fo, ws, stream);
    return SWSPH_OK;
}

int swsph_force_backward(swsph_plan* pl, const swsph_particles* p, const swsph_density_out* d,
                         const swsph_force_grad* g, swsph_input_grad* gi, void* ws, void* stream) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    int r = check_particles(pl, p, true);
    if (r) return r;
    if (!d || (p->n > 0 && (!d->h || !d->rho || !d->f || !d->rho_dh || !d->wcount || !d->wcount_dh)))
        return fail(SWSPH_E_ARG, "backward needs density h, rho, f, rho_dh, wcount, wcount_dh");
    if (!g || (p->n > 0 && (!g->gax || !g->gay || !g->gaz || !g->gdudt)))
        return fail(SWSPH_E_ARG, "backward needs dL/da and dL/d(du/dt)");
    if (!gi) return fail(SWSPH_E_ARG, "input gradient output is NULL");
    r = check_bound(pl, p, ws);
    if (r) return r;
    hipStream_t s = (hipStream_t)stream;
    BinPtrs b = ptrs_of(pl, ws);
    Scheme sc = scheme_of(pl);
    const int64_t n = b.n;
    void* dst[8] = {gi->gx, gi->gy, gi->gz, gi->gvx, gi->gvy, gi->gvz, gi->gu, gi->gm};
    const int src[8] = {7, 8, 9, 10, 11, 12, 14, 13};  // adjoint scratch arrays (binned order)
    if (pl->cfg.dtype == SWSPH_F64) {
        r = launch_backward<double>(b, sc, g, d, pl->lds_cap, s);
        for (int k = 0; k < 8; ++k)
            launch_unsort<double>(n, b.rank, (double*)b.adj + src[k] * adj_stride(n), dst[k], s);
    } else {
        r = launch_backward<float>(b, sc, g, d, pl->lds_cap, s);
        for (int k = 0; k < 8; ++k)
            launch_unsort<float>(n, b.rank, (float*)b.adj + src[k] * adj_stride(n), dst[k], s);
    }
    if (r) return fail(SWSPH_E_HIP, "backward kernel launch failed");
    return hip_check(hipGetLastError(), "force_backward");
}

int swsph_autotune(swsph_plan* pl, const swsph_particles* p, void* ws, void* stream,
                   const char* cache_path) {
    if (!pl) return fail(SWSPH_E_ARG, "plan is NULL");
    int r = check_particles(pl, p, true);
    if (r) return r;
    if (!ws) return fail(SWSPH_E_ARG, "workspace is NULL");
    if (pl->cfg.flags & SWSPH_PER_TASK_LAUNCH)
        return fail(SWSPH_E_ARG, "autotune times the batched launch; not for PER_TASK_LAUNCH");
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    hipDeviceProp_t prop;
    r = hip_check(hipGetDevice(&dev), "get device");
    if (r) return r;
    r = hip_check(hipGetDeviceProperties(&prop, dev), "device properties");
    if (r) return r;
    char key[640];
    snprintf(key, sizeof key, "%s|n=%lld|boxes=%d|dtype=%d|flags=%u", prop.gcnArchName,
             (long long)p->n, p->n_box, pl->cfg.dtype,
             pl->cfg.flags & (SWSPH_FIXED_H | SWSPH_NO_VISC | SWSPH_FLAT_LAUNCH));
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char line[1024];
            bool hit = false;
            while (std::fgets(line, sizeof line, f)) {
                char k2[640];
                int t = 0, td = 0, c = 0, cd = 0, o = 0, lm = 0;
                auto tile_ok = [](int v) { return v == 8 || v == 16 || v == 32 || v == 64; };
                auto cap_ok = [](int v) { return v == 128 || v == 256 || v == 512; };
                if (std::sscanf(line, "%639s %d %d %d %d %d %d", k2, &t, &td, &c, &cd, &o, &lm) ==
                        7 &&
                    std::strcmp(k2, key) == 0 && tile_ok(t) && tile_ok(td) && cap_ok(c) &&
                    cap_ok(cd) && (o == 0 || o == 1) && lm >= 1 && lm <= 4096) {
                    pl->tile = t;
                    pl->tile_d = td;
                    pl->lds_cap = c;
                    pl->lds_cap_d = cd;
                    pl->order = o;
                    pl->leaf_max = lm;
                    hit = true;
                }
            }
            std::fclose(f);
            if (hit) return SWSPH_OK;
        }
    }
    // The timed step writes its outputs into the adjoint region of the
    // workspace (free outside swsph_force_backward); sizes follow a bin.
    r = swsph_bin(pl, p, ws, stream);
    if (r) return r;
    const int64_t n = p->n;
    const uint64_t tsz = pl->cfg.dtype == SWSPH_F64 ? 8 : 4;
    char* a = (char*)ws + pl->G.lay.adj;
    auto arr = [&](int k) { return (void*)(a + (uint64_t)k * tsz * (uint64_t)n); };
    swsph_density_out d{arr(0), arr(1), arr(2), arr(3), arr(4), arr(5), arr(6), arr(7), arr(8),
                        arr(9), (int32_t*)arr(10), (int32_t*)arr(11)};
    swsph_gradient_out go{arr(12), arr(13)};
    swsph_force_out fo{arr(14), arr(15), arr(16), arr(17), (int32_t*)arr(18)};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    r = hip_check(hipEventCreate(&e0), "event");
    if (!r) r = hip_check(hipEventCreate(&e1), "event");
    auto time_one = [&](const int (&w)[6], float& best_ms) -> int {
        pl->tile = w[0];
        pl->tile_d = w[1];
        pl->lds_cap = w[2];
        pl->lds_cap_d = w[3];
        pl->order = w[4];
        pl->leaf_max = w[5];
        float ms = 3.0e38f;
        for (int rep = 0; rep < 2; ++rep) {
            int q = hip_check(hipEventRecord(e0, s), "event record");
            if (!q) q = swsph_step(pl, p, &d, &go, &fo, ws, stream);
            if (!q) q = hip_check(hipEventRecord(e1, s), "event record");
            if (!q) q = hip_check(hipEventSynchronize(e1), "event sync");
            if (q) return q;
            float t = 0.f;
            q = hip_check(hipEventElapsedTime(&t, e0, e1), "elapsed");
            if (q) return q;
            ms = std::min(ms, t);
        }
        swsph_stats st;
        const int q = swsph_read_stats(pl, ws, &st, stream);
        if (q) return q;
        best_ms = ms;
        return SWSPH_OK;
    };
    // coordinate descent over the options: gradient/force tile size, density
    // tile size, LDS capacities (gradient/force, density), task order, and
    // the cell size at which the task search stops splitting
    int v[6] = {pl->tile, pl->tile_d, pl->lds_cap, pl->lds_cap_d, pl->order, pl->leaf_max};
    float best = 3.0e38f;
    if (!r) r = time_one(v, best);
    const int tiles[4] = {8, 16, 32, 64}, caps[3] = {128, 256, 512}, orders[2] = {0, 1};
    const int leaves[3] = {16, 32, 64};
    const int* cand[6] = {tiles, tiles, caps, caps, orders, leaves};
    const int ncand[6] = {4, 4, 3, 3, 2, 3};
    for (int d = 0; d < 6 && !r; ++d) {
        for (int k = 0; k < ncand[d] && !r; ++k) {
            if (cand[d][k] == v[d]) continue;
            int w[6] = {v[0], v[1], v[2], v[3], v[4], v[5]};
            w[d] = cand[d][k];
            float t = 0.f;
            r = time_one(w, t);
            if (!r && t < best) {
                best = t;
                v[d] = w[d];
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    pl->tile = v[0];
    pl->tile_d = v[1];
    pl->lds_cap = v[2];
    pl->lds_cap_d = v[3];
    pl->order = v[4];
    pl->leaf_max = v[5];
    if (r) return r;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%s %d %d %d %d %d %d\n", key, v[0], v[1], v[2], v[3], v[4], v[5]);
            std::fclose(f);
        }
    }
    // leave the workspace binned with the chosen tiles
    return swsph_bin(pl, p, ws, stream);
}

}  // extern "C"
