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
    int32_t n_tiles;
    const int32_t* cstart;
    const float* hpyr;
    const T* hs;
    int32_t* leaf_cnt;
    const int32_t* leaf_off;
    int2* leaves;
    int64_t leaf_cap;
    float* trad;
    const int32_t* tflag;
    Counters* cnt;
    T eps;
    T margin;
    int32_t leaf_max;
};

// MODE: 0 density (radius eps*hmax*margin), 1 gradient (eps*hmax),
// 2 force (eps*hmax, and cells whose own support reaches the tile).
template <typename T, int MODE>
__global__ void __launch_bounds__(TASK_WPB * WAVE) k_tasks(TArgs<T> a, int pass, int fixup) {
    __shared__ SearchMem smem_search[TASK_WPB];
    const int wave = threadIdx.x / WAVE;
    const int t = blockIdx.x * TASK_WPB + wave;
    if (t >= a.n_tiles) return;
    SearchMem& m = smem_search[wave];
    const int lane = lane_id();
    const Tile tl = a.tiles[t];
    const bool skip = tl.count <= 0 || (fixup && a.tflag[t] == 0);
    if (skip) {
        if (pass == 0 && lane == 0) {
            a.leaf_cnt[t] = 0;
            if (!fixup) a.trad[t] = 0.f;
        }
        return;
    }
    const BoxInfo bi = a.boxtab[tl.box];
    const float L = (float)bi.L;
    const float Rcap = 0.5f * L * (1.0f - 1e-6f);
    float R;
    if (pass == 1 || (MODE == 0 && fixup)) {
        R = a.trad[t];
    } else {
        const bool act = lane < tl.count;
        const T h = act ? a.hs[tl.begin + lane] : (T)0;
        const T hmax = wave_max(h);
        R = (float)(a.eps * hmax * a.margin);
        if (!(R < Rcap)) {
            if (MODE != 0 && lane == 0) latch(a.cnt, SWSPH_ST_REACH);
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
    search_init(m, st, bi, g, Rstart);
    const float R2 = R * R;
    int64_t total = 0, cand = 0;
    const int64_t base = pass == 1 ? (int64_t)a.leaf_off[t] : 0;
    const int64_t mine = pass == 1 ? (int64_t)a.leaf_cnt[t] : 0;
    for (int guard = 0; guard < SEARCH_MAX_CHUNKS; ++guard) {
        const bool done = search_step<MODE == 2>(m, st, bi, g, R2, a.cstart, a.hpyr, a.leaf_max,
                                                 a.cnt);
        if (st.nleaf > 0) {
            if (pass == 1) {
                for (int k = lane; k < st.nleaf; k += WAVE) {
                    const int64_t at = total + k;
                    if (at < mine && base + at < a.leaf_cap)
                        a.leaves[base + at] = pack_leaf(m.lbeg[k], m.lcnt[k], m.lshift[k]);
                }
            } else {
                int c = 0;
                for (int k = lane; k < st.nleaf; k += WAVE) c += m.lcnt[k];
                cand += wave_sum(c);
            }
            total += st.nleaf;
            st.nleaf = 0;
            wave_sync();
        }
        if (done) break;
    }
    if (lane == 0) {
        if (pass == 0) {
            a.leaf_cnt[t] = (int32_t)total;
            a.tiles[t].cost = (float)tl.count * (float)cand;
            atomicAdd(&a.cnt->leaves, (unsigned long long)total);
        } else if (base + total > a.leaf_cap) {
            latch(a.cnt, SWSPH_ST_CAPACITY);
        }
    }
}

template <typename T>
static TArgs<T> targs(const BinPtrs& b, const Scheme& sc, double margin) {
    TArgs<T> a;
    a.boxtab = b.boxtab;
    a.tiles = b.tiles;
    a.n_tiles = b.n_tiles;
    a.cstart = b.cstart;
    a.hpyr = b.hmaxpyr;
    a.hs = (const T*)b.hs;
    a.leaf_cnt = b.leaf_cnt;
    a.leaf_off = b.leaf_off;
    a.leaves = b.leaves;
    a.leaf_cap = b.leaf_cap;
    a.trad = b.trad;
    a.tflag = b.tflag;
    a.cnt = b.cnt;
    a.eps = (T)sc.eps;
    a.margin = (T)margin;
    a.leaf_max = sc.leaf_max;
    return a;
}

template <typename T>
void launch_tasks(const BinPtrs& b, const Scheme& sc, int mode, bool fixup, hipStream_t s) {
    if (b.n_tiles <= 0) return;
    const double margin = (mode == 0 && !(sc.flags & SWSPH_FIXED_H)) ? 1.25 : 1.0;
    TArgs<T> a = targs<T>(b, sc, margin);
    const dim3 grid((unsigned)((b.n_tiles + TASK_WPB - 1) / TASK_WPB)), block(TASK_WPB * WAVE);
    void (*kern)(TArgs<T>, int, int) =
        mode == 0 ? k_tasks<T, 0> : (mode == 1 ? k_tasks<T, 1> : k_tasks<T, 2>);
    auto run = [&](int pass) {
        hipLaunchKernelGGL(kern, grid, block, 0, s, a, pass, (int)fixup);
    };
    run(0);
    launch_exclusive_scan(b.leaf_cnt, b.n_tiles, b.leaf_part, b.leaf_off, s);
    run(1);
}
template void launch_tasks<float>(const BinPtrs&, const Scheme&, int, bool, hipStream_t);
template void launch_tasks<double>(const BinPtrs&, const Scheme&, int, bool, hipStream_t);

}  // namespace swsph
