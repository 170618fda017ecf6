// tasks.hip -- device task lists: for every i-tile, the candidate
// j-particles its loop must visit (from the recursive cell search of
// search.h, culled against the tile box), stored as cand_off[t] ..
// cand_off[t] + cand_cnt[t] in `cands`.  One search per tile; lists are
// contiguous per tile and placed by a bump counter (their content and order
// do not depend on the placement).  The build also fixes the tile's search
// radius (trad), which the loop kernels reuse, and a cost estimate (tile
// particles x candidates) for task ordering.
#include <algorithm>

#include "launch.h"
#include "search.h"

namespace swsph {

constexpr int TASK_WPB = 4;

template <typename T>
struct TArgs {
    const BoxInfo* boxtab;
    Tile* tiles;
    const unsigned long long* ntiles;
    int64_t tile_cap;
    const int32_t* cstart;
    const float* hpyr;
    const T* hs;
    int32_t* cand_cnt;
    int32_t* cand_off;
    uint32_t* cands;
    int64_t cand_cap;
    float* trad;
    const int32_t* tflag;
    float* fbox;  // density fix-ups: box of each flagged tile's pending particles
    Counters* cnt;
    T eps;
    T margin;   // on the tile's radius eps * hmax
    T hmargin;  // force: on every particle's support H_j (and the cell maxima)
    int32_t leaf_max;
    const V4<T>* pos4;
    int64_t n;
    const int32_t* list;  // tiles to build (first *ntiles entries), or null: every tile
    unsigned long long* heads;  // item-queue heads (NSEG, zeroed before the launch)
};

// Task list of tile t: its candidate j-particles -- the particles of the
// cells the cell search keeps whose distance to the tile's bounding box is
// below the loop's radius R (force: below max(R, H_j), the symmetric
// support) -- as entries j | image << 26 (periodic image code, see
// search.h).  The cull is done once here, so the loops only gather.
// Each wavefront owns a window of the candidate array, TASK_CHUNK entries
// taken from a device bump counter, and writes its tiles' lists into it one
// after another, straight to their final place (no staging buffer, no copy):
// a tile starts with at least TASK_BUF free entries in the window, and a
// list that turns out longer is counted, given exactly that much space from
// the same counter, and the search runs again writing there.  Lists stay
// contiguous; the window's unused tail is left as a gap.  The tile's radius
// and cost (particles x candidates) are recorded.  Wavefront-uniform.
constexpr int TASK_BUF = 2048;     // longest list written in one search
static_assert(TASK_CHUNK >= TASK_BUF, "a window must hold the longest single-search list");

struct TaskMem {
    SearchMem sm;
    int32_t lpre[LEAFCAP + 1];  // prefix sums of the particle counts of a leaf batch
};

// The wavefront's window [at, end) of the candidate array.
struct TaskWindow {
    int64_t at = 0, end = 0;
};

// The particles of a batch of leaves (cell ranges with image codes, their
// counts' prefix sums in lpre), visited in order, WAVE x U at a time: the
// particle index of every slot is found first and all their loads are issued
// together, so a wavefront waits for one memory round trip per U x 64
// candidates instead of one per 64.  visit(have, j, code, pos, h_j) is called
// by the whole wavefront (it may ballot); lanes past the end get have=false.
constexpr int CAND_U = 16;

template <typename T, bool NEEDH, typename F>
__device__ __forceinline__ void for_candidates(const SearchMem& sm, const int32_t* lpre, int nl,
                                               int nv, const V4<T>* __restrict__ pos4,
                                               const T* __restrict__ hs, int64_t n, F&& visit) {
    const int lane = lane_id();
    int top = 1;  // largest power of two <= nl (uniform)
    while (2 * top <= nl) top *= 2;
    for (int v0 = 0; v0 < nv; v0 += CAND_U * WAVE) {
        // leaf of slot v: the last leaf whose prefix is <= v (prefixes rise
        // strictly, lpre[0] = 0, lpre[nl..2 WAVE] = the total), by binary
        // lifting with a uniform step count so the slots' LDS reads overlap
        int lo[CAND_U];
#pragma unroll
        for (int u = 0; u < CAND_U; ++u) lo[u] = 0;
        for (int st = top; st > 0; st >>= 1) {
            // unconditional reads (no branch around them, so they overlap):
            // prefixes from nl on equal the total and never pass the test
#pragma unroll
            for (int u = 0; u < CAND_U; ++u) {
                const int c = lo[u] + st;
                const int cr = c < 2 * WAVE ? c : 2 * WAVE;
                lo[u] = lpre[cr] <= v0 + u * WAVE + lane ? c : lo[u];
            }
        }
        int jj[CAND_U], cc[CAND_U];
#pragma unroll
        for (int u = 0; u < CAND_U; ++u) {
            const int v = v0 + u * WAVE + lane;
            jj[u] = 0;
            cc[u] = 0;
            if (v < nv) {
                const int j = sm.lbeg[lo[u]] + (v - lpre[lo[u]]);
                jj[u] = (j < 0 || j >= (int)n) ? 0 : j;  // cannot happen with a valid cell table
                cc[u] = sm.lshift[lo[u]];
            }
        }
        V4<T> pa[CAND_U];
        T hj[CAND_U];
#pragma unroll
        for (int u = 0; u < CAND_U; ++u) pa[u] = pos4[jj[u]];
#pragma unroll
        for (int u = 0; u < CAND_U; ++u) hj[u] = NEEDH ? hs[jj[u]] : (T)0;
#pragma unroll
        for (int u = 0; u < CAND_U; ++u) {
            if (v0 + u * WAVE >= nv) break;  // uniform
            visit(v0 + u * WAVE + lane < nv, jj[u], cc[u], pa[u], hj[u]);
        }
    }
}

// Returns the number of entries listed for the tile (uniform over the wave).
template <typename T, int MODE>
__device__ int64_t task_one(const TArgs<T>& a, TaskMem& m, TaskWindow& win, const Tile& tl,
                            int64_t t, int fixup) {
    const int lane = lane_id();
    if (win.end - win.at < TASK_BUF) {
        // a new window; none left -> the capacity error below
        int64_t w = 0;
        if (lane == 0) {
            w = (int64_t)atomicAdd(&a.cnt->cand_used, (unsigned long long)TASK_CHUNK);
            if (w + TASK_CHUNK > a.cand_cap) w = -1;
        }
        w = __shfl(w, 0, WAVE);
        win.at = w;
        win.end = w < 0 ? w : w + TASK_CHUNK;
    }
    const bool room = win.at >= 0;
    const BoxInfo bi = a.boxtab[tl.box];
    const float L = (float)bi.L;
    const float Rcap = 0.5f * L * (1.0f - 1e-6f);
    float R;
    if (MODE == 0 && fixup) {
        R = a.trad[t];
    } else {
        const bool act = lane < tl.count;
        // (a density fix-up marks a pending h by its sign)
        const T h = act ? fabs(a.hs[tl.begin + lane]) : (T)0;
        const T hmax = wave_max(h);
        // float radius rounded up so it still covers every support of the tile
        R = (float)(a.eps * hmax * a.margin * (T)(1 + 4e-7));
        if (!(R < Rcap)) {
            // fixed supports (every loop but the Newton density search) must fit
            if (a.margin == (T)1 && lane == 0) latch(a.cnt, SWSPH_ST_REACH);
            R = Rcap;
        }
        if (!(R > 0.f)) R = Rcap;
        if (lane == 0) a.trad[t] = R;
    }
    TileGeom g;
#pragma unroll
    for (int d = 0; d < 3; ++d) { g.lo[d] = tl.lo[d]; g.hi[d] = tl.hi[d]; }
    if (MODE == 0 && fixup && a.fbox) {
        // a density fix-up iterates only the particles left pending (their
        // h stored negated): the list serves the box around them, which is
        // recorded for the loop (it culls with the same box)
        const bool pend = lane < tl.count && a.hs[tl.begin + lane] < (T)0;
        if (ballot(pend) != 0ull) {
            const V4<T> p = a.pos4[tl.begin + (pend ? lane : 0)];
            const T big = (T)3.0e38f;
            const T px[3] = {p.x, p.y, p.z};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                g.lo[d] = float_down(wave_min(pend ? px[d] : big));
                g.hi[d] = float_up(wave_max(pend ? px[d] : -big));
            }
            if (lane == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    a.fbox[6 * t + d] = g.lo[d];
                    a.fbox[6 * t + 3 + d] = g.hi[d];
                }
            }
        }
    }
    float Rstart = R;
    const float hm = (float)a.hmargin;
    if (MODE == 2) Rstart = fmaxf(R, a.hpyr[bi.pyr_off] * hm);
    const float R2 = R * R;
    const T Rt = (T)R;
    const T R2t = Rt * Rt;  // the loops cull with the same value
    const T Lt = (T)bi.L;
    bool direct = false;    // second round: write to global memory at base
    int64_t base = 0, known = 0, listed = 0;
    for (int round = 0; round < 2; ++round) {
        SearchState st;
        search_init(m.sm, st, bi, g, Rstart);
        int64_t total = 0;
        for (int guard = 0; guard < SEARCH_MAX_CHUNKS; ++guard) {
            const bool done = search_step<MODE == 2>(m.sm, st, bi, g, R2, a.cstart, a.hpyr, hm,
                                                     a.leaf_max, a.cnt);
            if (st.nleaf > 0) {
                // prefix sums of the batch's particle counts (two lanes' worth each)
                int c0 = lane < st.nleaf ? m.sm.lcnt[lane] : 0;
                int c1 = lane + WAVE < st.nleaf ? m.sm.lcnt[lane + WAVE] : 0;
                int tot0 = 0, tot1 = 0;
                const int e0 = wave_excl_scan(c0, tot0);
                const int e1 = wave_excl_scan(c1, tot1);
                m.lpre[lane] = e0;
                m.lpre[lane + WAVE] = tot0 + e1;
                if (lane == 0) m.lpre[2 * WAVE] = tot0 + tot1;
                wave_sync();
                const int nl = st.nleaf;
                const int nv = tot0 + tot1;
                for_candidates<T, MODE == 2>(
                    m.sm, m.lpre, nl, nv, a.pos4, a.hs, a.n,
                    [&](bool have, int j, int code, const V4<T>& pa, T hj) {
                        bool pass = false;
                        uint32_t ent = 0;
                        if (have) {
                            int sx, sy, sz;
                            shift_of(code, sx, sy, sz);
                            const T xs = pa.x + (T)sx * Lt, ys = pa.y + (T)sy * Lt,
                                    zs = pa.z + (T)sz * Lt;
                            const T gx = max((T)0, max((T)g.lo[0] - xs, xs - (T)g.hi[0]));
                            const T gy = max((T)0, max((T)g.lo[1] - ys, ys - (T)g.hi[1]));
                            const T gz = max((T)0, max((T)g.lo[2] - zs, zs - (T)g.hi[2]));
                            const T d2 = dist2_unfused(gx, gy, gz);
                            T crit = R2t;
                            if (MODE == 2) {
                                const T Hj = mul_unfused(a.eps, hj) * a.hmargin;
                                crit = max(crit, mul_unfused(Hj, Hj));
                            }
                            pass = d2 < crit;
                            ent = (uint32_t)j | ((uint32_t)code << 26);
                        }
                        const unsigned long long pm = ballot(pass);
                        if (pass) {
                            const int64_t at = total + mbcnt(pm);
                            if (direct) {
                                if (at < known) a.cands[base + at] = ent;
                            } else if (room && at < TASK_BUF) {
                                a.cands[win.at + at] = ent;
                            }
                        }
                        total += __popcll(pm);
                    });
                st.nleaf = 0;
                wave_sync();
            }
            if (done) break;
        }
        if (direct) break;
        // first round: a list that fit is in place in the window; a longer
        // one gets exact space (or the capacity error) and a second round
        int64_t at = 0;
        listed = total;
        const bool inwin = room && total <= TASK_BUF;
        if (lane == 0) {
            a.tiles[t].cost = (float)tl.count * (float)total;
            if (inwin) {
                at = win.at;
            } else if (room) {
                at = (int64_t)atomicAdd(&a.cnt->cand_used, (unsigned long long)total);
                if (at + total > a.cand_cap) at = -1;
            } else {
                at = -1;
            }
            a.cand_off[t] = at >= 0 ? (int32_t)at : -1;
            a.cand_cnt[t] = at >= 0 ? (int32_t)total : 0;
            if (at < 0) latch(a.cnt, SWSPH_ST_CAPACITY);
        }
        at = __shfl(at, 0, WAVE);
        if (inwin) {
            win.at += total;
            break;
        }
        if (at < 0) break;
        direct = true;
        base = at;
        known = total;
        wave_sync();
    }
    wave_sync();
    return listed;
}

// MODE: 0 density (radius eps*hmax*margin), 1 gradient (eps*hmax),
// 2 force (eps*hmax, and cells whose own support reaches the tile).
// One wavefront per tile; tiles are popped from the item queue (for_each_item).
// The builds wait on dependent loads: 16 x 64 candidate loads in flight per
// wavefront hide more of that than more wavefronts with fewer loads each, so
// the register budget allows three wavefronts per SIMD (two for the force
// build, which also loads h_j) and no spills.
template <typename T, int MODE>
__global__ void __launch_bounds__(TASK_WPB * WAVE)
SWSPH_WAVES_PER_EU(sizeof(T) != 4 ? 1 : (MODE == 2 ? 2 : 3)) k_tasks(TArgs<T> a, int fixup) {
    __shared__ TaskMem smem_task[TASK_WPB];
    const int wave = threadIdx.x / WAVE;
    TaskMem& m = smem_task[wave];
    const int lane = lane_id();
    const int64_t nt = (int64_t)*a.ntiles;
    unsigned long long listed = 0;  // flushed once per wavefront
    TaskWindow win;
    for_each_item(a.heads, nt, a.list == nullptr, [&](int64_t k) {
        const int64_t t = a.list ? (int64_t)uniform(a.list[k]) : k;
        Tile tl = a.tiles[t];
        tl.count = uniform(tl.count);
        tl.box = uniform(tl.box);
        const bool skip = tl.count <= 0 || (fixup && a.tflag[t] == 0);
        if (skip) {
            if (lane == 0) {
                a.cand_cnt[t] = 0;
                if (!fixup) a.trad[t] = 0.f;
            }
            return;
        }
        listed += (unsigned long long)task_one<T, MODE>(a, m, win, tl, t, fixup);
    });
    if (lane == 0 && listed) atomicAdd(&a.cnt->listed, listed);
}

// Queue order of the tiles by decreasing cost (longest task first), so the
// persistent kernel does not end on a few large tasks.  A stable counting
// sort on 32 logarithmic cost classes: blocks own contiguous runs of
// ORD_T x ORD_I tiles and threads contiguous runs of ORD_I, so equal classes
// keep tile order and the result is deterministic.  Three launches: per
// block class histograms, a scan of the class-major table, the scatter.
constexpr int ORD_T = 256, ORD_I = 8, ORD_B = 32;
constexpr int ORD_CHUNK = ORD_T * ORD_I;

__device__ __forceinline__ int cost_class(float c) {
    int e = 0;
    if (c >= 1.f) frexpf(c, &e);                      // c in [2^(e-1), 2^e)
    return max(0, min(ORD_B - 1, ORD_B - 1 - e));     // large cost -> small class
}

// Per-thread class counts of the block's tiles, exclusive over the block's
// threads (hist[c][k] = tiles of class c before thread k's run).
__device__ __forceinline__ void block_class_counts(const Tile* __restrict__ tiles, int64_t nt,
                                                   int32_t (&hist)[ORD_B][ORD_T],
                                                   int32_t (&tot)[ORD_B], int64_t& lo,
                                                   int64_t& hi) {
    const int k = threadIdx.x;
    lo = min(nt, (int64_t)blockIdx.x * ORD_CHUNK + (int64_t)k * ORD_I);
    hi = min(nt, lo + ORD_I);
    for (int c = 0; c < ORD_B; ++c) hist[c][k] = 0;
    for (int64_t t = lo; t < hi; ++t) ++hist[cost_class(tiles[t].cost)][k];
    __syncthreads();
    if (k < ORD_B) {
        int run = 0;
        for (int j = 0; j < ORD_T; ++j) {
            const int v = hist[k][j];
            hist[k][j] = run;
            run += v;
        }
        tot[k] = run;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(ORD_T) k_order_hist(const Tile* __restrict__ tiles,
                                                      const unsigned long long* __restrict__ ntiles,
                                                      int32_t nblk, int32_t* __restrict__ table) {
    __shared__ int32_t hist[ORD_B][ORD_T];
    __shared__ int32_t tot[ORD_B];
    const int64_t nt = (int64_t)*ntiles;
    int64_t lo, hi;
    block_class_counts(tiles, nt, hist, tot, lo, hi);
    if (threadIdx.x < ORD_B) table[(int64_t)threadIdx.x * nblk + blockIdx.x] = tot[threadIdx.x];
}

__global__ void __launch_bounds__(ORD_T) k_order_scatter(const Tile* __restrict__ tiles,
                                                         const unsigned long long* __restrict__ ntiles,
                                                         int32_t nblk,
                                                         const int32_t* __restrict__ base,
                                                         int32_t* __restrict__ order) {
    __shared__ int32_t hist[ORD_B][ORD_T];
    __shared__ int32_t tot[ORD_B];
    const int64_t nt = (int64_t)*ntiles;
    int64_t lo, hi;
    block_class_counts(tiles, nt, hist, tot, lo, hi);
    const int k = threadIdx.x;
    for (int64_t t = lo; t < hi; ++t) {
        const int c = cost_class(tiles[t].cost);
        order[base[(int64_t)c * nblk + blockIdx.x] + hist[c][k]++] = (int32_t)t;
    }
}

int64_t order_table_size(int64_t tile_cap) {
    return (int64_t)ORD_B * ((tile_cap + ORD_CHUNK - 1) / ORD_CHUNK) + 1;
}

void launch_order(const BinPtrs& b, hipStream_t s) {
    const int32_t nblk = (int32_t)((b.tile_cap + ORD_CHUNK - 1) / ORD_CHUNK);
    const int64_t nent = (int64_t)ORD_B * nblk;
    hipLaunchKernelGGL(k_order_hist, dim3(nblk), dim3(ORD_T), 0, s, (const Tile*)b.tiles,
                       (const unsigned long long*)b.ntiles, nblk, b.ord_table);
    launch_exclusive_scan(b.ord_table, nent, b.scan_part, b.ord_base, s);
    hipLaunchKernelGGL(k_order_scatter, dim3(nblk), dim3(ORD_T), 0, s, (const Tile*)b.tiles,
                       (const unsigned long long*)b.ntiles, nblk, (const int32_t*)b.ord_base,
                       b.order);
}

template <typename T>
static TArgs<T> targs(const BinPtrs& b, const Scheme& sc, double margin);

// Resident workgroups of a build kernel (items are popped, so a larger grid
// only adds empty pops).
static unsigned resident_grid(const void* kern, int threads) {
    static const void* keys[16];
    static unsigned vals[16];
    for (int i = 0; i < 16; ++i)
        if (keys[i] == kern) return vals[i];
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const unsigned g = (unsigned)(per_cu * device_cu_count());
    for (int i = 0; i < 16; ++i)
        if (!keys[i]) {
            keys[i] = kern;
            vals[i] = g;
            break;
        }
    return g;
}

template <typename T>
static TArgs<T> targs(const BinPtrs& b, const Scheme& sc, double margin) {
    TArgs<T> a;
    a.boxtab = b.boxtab;
    a.tiles = b.tiles;
    a.ntiles = b.ntiles;
    a.tile_cap = b.tile_cap;
    a.cstart = b.cstart;
    a.hpyr = b.hmaxpyr;
    a.hs = (const T*)b.hs;
    a.cand_cnt = b.cand_cnt;
    a.cand_off = b.cand_off;
    a.cands = b.cands;
    a.cand_cap = b.cand_cap;
    a.trad = b.trad;
    a.tflag = b.tflag;
    a.fbox = b.fbox;
    a.cnt = b.cnt;
    a.eps = (T)sc.eps;
    a.margin = (T)margin;
    a.hmargin = (T)1;
    a.leaf_max = sc.leaf_max;
    a.pos4 = (const V4<T>*)b.pos4;
    a.n = b.n;
    a.list = nullptr;
    a.heads = b.cnt->build_queue;
    return a;
}

template <typename T>
void launch_tasks(const BinPtrs& b, const Scheme& sc, int mode, bool fixup, hipStream_t s) {
    if (b.n <= 0) return;
    const bool guessed = (mode == 0 || mode == 3) && !(sc.flags & SWSPH_FIXED_H);
    const double margin = guessed ? (mode == 3 ? SINGLE_MARGIN : DENS_MARGIN) : 1.0;
    TArgs<T> a = targs<T>(b, sc, margin);
    if (mode == 3) {
        // the force loop's lists before h is known: every support at the
        // density margin over its guess (supersets of the lists at the final
        // h wherever no h ends beyond that margin)
        a.hmargin = (T)margin;
        mode = 2;
    }
    // the density builds stop refining at 8x larger cells: their search (a
    // chain of dependent cell-table loads, most of the build's time) gets
    // shallower and the walk over the leaves' particles, which culls each
    // one exactly, costs less than the levels it saves; the force build,
    // whose cells also pass on their largest support, keeps leaf_max
    if (mode == 0) a.leaf_max = std::min(sc.leaf_max * 8, 4096);
    if (fixup) {
        // the flagged tiles (b.tflag), compacted into b.tmpidx
        a.list = b.tmpidx;
        a.ntiles = &b.cnt->n_fix;
    }
    const dim3 block(TASK_WPB * WAVE);
    void (*kern)(TArgs<T>, int) =
        mode == 0 ? k_tasks<T, 0> : (mode == 1 ? k_tasks<T, 1> : k_tasks<T, 2>);
    launch_fill_u32(&b.cnt->cand_used, 2, 0u, s);
    launch_fill_u32(a.heads, 2 * NSEG, 0u, s);
    // at most b.build_waves wavefronts take windows (the candidate capacity
    // counts on it)
    const unsigned gmax = (unsigned)std::max<int64_t>(1, b.build_waves / TASK_WPB);
    const unsigned grid = std::min(resident_grid((const void*)kern, TASK_WPB * WAVE), gmax);
    hipLaunchKernelGGL(kern, dim3(grid), block, 0, s, a,
                       (int)fixup);
    if (!fixup && sc.order == 0) launch_order(b, s);
}
template void launch_tasks<float>(const BinPtrs&, const Scheme&, int, bool, hipStream_t);
template void launch_tasks<double>(const BinPtrs&, const Scheme&, int, bool, hipStream_t);

}  // namespace swsph
