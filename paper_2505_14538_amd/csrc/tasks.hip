// tasks.hip -- device task lists: for every i-tile, the cells (leaves of the
// recursive cell search, see search.h) its loop must visit, stored as a CSR:
// leaf_off[t] .. leaf_off[t] + leaf_cnt[t] in `leaves`.
//
// Built in two passes (count, then fill after an exclusive scan of the
// counts) so the list needs no atomics and comes out in a fixed order.  The
// count pass also fixes the tile's search radius (trad), which the loop
// kernels reuse for their per-particle cull, and a cost estimate
// (tile particles x candidate particles) for task ordering.
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
    int32_t* leaf_cnt;
    int32_t* leaf_off;
    int2* leaves;
    int64_t leaf_cap;
    float* trad;
    const int32_t* tflag;
    int32_t* ovf;               // tiles whose list overflowed the LDS buffer
    Counters* cnt;
    T eps;
    T margin;
    int32_t leaf_max;
};

// Task list of tile t from one cell search.  Main pass: the tile's leaves
// are gathered in LDS (up to TASK_BUF) and copied to space taken from a
// device bump counter, so each tile's list is contiguous; its radius and
// cost are recorded.  A tile with more leaves only counts them and is put
// on the overflow list; the overflow pass takes exactly that much space and
// runs its search again, writing straight to global memory.
// Wavefront-uniform.
#ifndef SWSPH_TASK_BUF
#define SWSPH_TASK_BUF 512
#endif
constexpr int TASK_BUF = SWSPH_TASK_BUF;  // leaves buffered in LDS per wavefront

struct TaskMem {
    SearchMem sm;
    int2 buf[TASK_BUF];
};

template <typename T, int MODE>
__device__ void task_one(const TArgs<T>& a, TaskMem& m, const Tile& tl, int64_t t,
                         bool overflow_pass, int fixup, int64_t base) {
    const int lane = lane_id();
    const BoxInfo bi = a.boxtab[tl.box];
    const float L = (float)bi.L;
    const float Rcap = 0.5f * L * (1.0f - 1e-6f);
    float R;
    if (overflow_pass || (MODE == 0 && fixup)) {
        R = a.trad[t];
    } else {
        const bool act = lane < tl.count;
        const T h = act ? a.hs[tl.begin + lane] : (T)0;
        const T hmax = wave_max(h);
        // float radius rounded up so it still covers every support of the tile
        R = (float)(a.eps * hmax * a.margin * (T)(1 + 4e-7));
        if (!(R < Rcap)) {
            // fixed supports (every loop but the Newton density search) must fit
            if ((MODE != 0 || a.margin == (T)1) && lane == 0) latch(a.cnt, SWSPH_ST_REACH);
            R = Rcap;
        }
        if (!(R > 0.f)) R = Rcap;
        if (lane == 0) a.trad[t] = R;
    }
    TileGeom g;
#pragma unroll
    for (int d = 0; d < 3; ++d) { g.lo[d] = tl.lo[d]; g.hi[d] = tl.hi[d]; }
    float Rstart = R;
    if (MODE == 2) Rstart = fmaxf(R, a.hpyr[bi.pyr_off]);
    SearchState st;
    search_init(m.sm, st, bi, g, Rstart);
    const float R2 = R * R;
    int64_t total = 0, cand = 0;
    const int64_t mine = overflow_pass ? (int64_t)a.leaf_cnt[t] : 0;
    for (int guard = 0; guard < SEARCH_MAX_CHUNKS; ++guard) {
        const bool done = search_step<MODE == 2>(m.sm, st, bi, g, R2, a.cstart, a.hpyr,
                                                 a.leaf_max, a.cnt);
        if (st.nleaf > 0) {
            int c = 0;
            for (int k = lane; k < st.nleaf; k += WAVE) {
                const int64_t at = total + k;
                const int2 v = pack_leaf(m.sm.lbeg[k], m.sm.lcnt[k], m.sm.lshift[k]);
                if (overflow_pass) {
                    if (at < mine && base + at < a.leaf_cap) a.leaves[base + at] = v;
                } else if (at < TASK_BUF) {
                    m.buf[at] = v;
                }
                c += m.sm.lcnt[k];
            }
            cand += wave_sum(c);
            total += st.nleaf;
            st.nleaf = 0;
            wave_sync();
        }
        if (done) break;
    }
    if (!overflow_pass) {
        int64_t at = 0;
        if (lane == 0) {
            a.leaf_cnt[t] = (int32_t)total;
            a.tiles[t].cost = (float)tl.count * (float)cand;
            atomicAdd(&a.cnt->leaves, (unsigned long long)total);
            if (total > TASK_BUF) {
                a.leaf_off[t] = -1;
                a.ovf[atomicAdd(&a.cnt->n_ovf, 1ull)] = (int32_t)t;
            } else {
                at = (int64_t)atomicAdd(&a.cnt->leaf_used, (unsigned long long)total);
                a.leaf_off[t] = at + total <= a.leaf_cap ? (int32_t)at : -1;
                if (at + total > a.leaf_cap) {
                    a.leaf_cnt[t] = 0;
                    latch(a.cnt, SWSPH_ST_CAPACITY);
                }
            }
        }
        at = __shfl(at, 0, WAVE);
        if (total <= TASK_BUF && at + total <= a.leaf_cap)
            for (int k = lane; k < total; k += WAVE) a.leaves[at + k] = m.buf[k];
    } else if (lane == 0 && base + total > a.leaf_cap) {
        latch(a.cnt, SWSPH_ST_CAPACITY);
    }
    wave_sync();
}

// MODE: 0 density (radius eps*hmax*margin), 1 gradient (eps*hmax),
// 2 force (eps*hmax, and cells whose own support reaches the tile).
// One wavefront per tile, grid-stride over the device tile count.
template <typename T, int MODE>
__global__ void __launch_bounds__(TASK_WPB * WAVE) k_tasks(TArgs<T> a, int fixup) {
    __shared__ TaskMem smem_task[TASK_WPB];
    const int wave = threadIdx.x / WAVE;
    TaskMem& m = smem_task[wave];
    const int lane = lane_id();
    const int64_t nt = (int64_t)*a.ntiles;
    const int64_t nw = (int64_t)gridDim.x * TASK_WPB;
    for (int64_t t = blockIdx.x * (int64_t)TASK_WPB + wave; t < nt; t += nw) {
        Tile tl = a.tiles[t];
        tl.count = uniform(tl.count);
        tl.box = uniform(tl.box);
        const bool skip = tl.count <= 0 || (fixup && a.tflag[t] == 0);
        if (skip) {
            if (lane == 0) {
                a.leaf_cnt[t] = 0;
                if (!fixup) a.trad[t] = 0.f;
            }
            continue;
        }
        task_one<T, MODE>(a, m, tl, t, false, fixup, 0);
    }
}

// Tiles whose list did not fit the LDS buffer: space of the counted size,
// then the search again.
template <typename T, int MODE>
__global__ void __launch_bounds__(TASK_WPB * WAVE) k_tasks_ovf(TArgs<T> a, int fixup) {
    __shared__ TaskMem smem_task[TASK_WPB];
    const int wave = threadIdx.x / WAVE;
    TaskMem& m = smem_task[wave];
    const int64_t no = (int64_t)a.cnt->n_ovf;
    const int64_t nw = (int64_t)gridDim.x * TASK_WPB;
    for (int64_t q = blockIdx.x * (int64_t)TASK_WPB + wave; q < no; q += nw) {
        const int64_t t = a.ovf[q];
        Tile tl = a.tiles[t];
        tl.count = uniform(tl.count);
        tl.box = uniform(tl.box);
        int64_t at = 0;
        if (lane_id() == 0) {
            const int64_t c = a.leaf_cnt[t];
            at = (int64_t)atomicAdd(&a.cnt->leaf_used, (unsigned long long)c);
            if (at + c > a.leaf_cap) {
                a.leaf_cnt[t] = 0;
                latch(a.cnt, SWSPH_ST_CAPACITY);
                at = -1;
            }
            a.leaf_off[t] = (int32_t)at;
        }
        at = __shfl(at, 0, WAVE);
        if (at < 0) continue;
        task_one<T, MODE>(a, m, tl, t, true, fixup, at);
    }
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
static TArgs<T> targs(const BinPtrs& b, const Scheme& sc, double margin) {
    TArgs<T> a;
    a.boxtab = b.boxtab;
    a.tiles = b.tiles;
    a.ntiles = b.ntiles;
    a.tile_cap = b.tile_cap;
    a.cstart = b.cstart;
    a.hpyr = b.hmaxpyr;
    a.hs = (const T*)b.hs;
    a.leaf_cnt = b.leaf_cnt;
    a.leaf_off = b.leaf_off;
    a.leaves = b.leaves;
    a.leaf_cap = b.leaf_cap;
    a.trad = b.trad;
    a.tflag = b.tflag;
    a.ovf = b.ovf;
    a.cnt = b.cnt;
    a.eps = (T)sc.eps;
    a.margin = (T)margin;
    a.leaf_max = sc.leaf_max;
    return a;
}

template <typename T>
void launch_tasks(const BinPtrs& b, const Scheme& sc, int mode, bool fixup, hipStream_t s) {
    if (b.n <= 0) return;
    const double margin = (mode == 0 && !(sc.flags & SWSPH_FIXED_H)) ? 1.25 : 1.0;
    TArgs<T> a = targs<T>(b, sc, margin);
    const dim3 block(TASK_WPB * WAVE);
    void (*kern)(TArgs<T>, int) =
        mode == 0 ? k_tasks<T, 0> : (mode == 1 ? k_tasks<T, 1> : k_tasks<T, 2>);
    void (*kovf)(TArgs<T>, int) =
        mode == 0 ? k_tasks_ovf<T, 0> : (mode == 1 ? k_tasks_ovf<T, 1> : k_tasks_ovf<T, 2>);
    launch_fill_u32(&b.cnt->leaf_used, 4, 0u, s);  // leaf_used and n_ovf
    hipLaunchKernelGGL(kern, dim3(wave_grid(b.tile_cap, TASK_WPB)), block, 0, s, a, (int)fixup);
    hipLaunchKernelGGL(kovf, dim3(wave_grid(1024, TASK_WPB)), block, 0, s, a, (int)fixup);
    if (!fixup && sc.order == 0) launch_order(b, s);
}
template void launch_tasks<float>(const BinPtrs&, const Scheme&, int, bool, hipStream_t);
template void launch_tasks<double>(const BinPtrs&, const Scheme&, int, bool, hipStream_t);

}  // namespace swsph
