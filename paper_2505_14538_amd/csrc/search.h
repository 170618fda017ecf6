// search.h -- recursive cell search of one i-tile over the implicit Morton
// cell tree of its box (device code, one wavefront per tile).
//
// The paper's solver builds self and pair tasks on cubic cells and recurses
// into daughter cells until a cell is about as wide as the search radius
// (Sec. 2.2.2).  Here a wavefront seeds its search with the cells of the
// coarsest level whose width is at least the search radius that overlap the
// tile's bounding box grown by that radius (periodic images included), keeps
// a cell while its distance to the tile box is below the radius (or, for the
// symmetric force loop, below the cell's own largest support radius), and
// splits a kept cell into its 8 children while it holds more than `leaf_max`
// particles and is not entirely within reach.  Kept cells that are not split
// ("leaves": one contiguous particle range each, with a periodic-image code)
// are handed out in batches; tasks.hip walks their particles.
//
// Every loop is bounded: the search processes at most SEARCH_MAX_CHUNKS
// chunks per call and latches SWSPH_ST_LOOPCAP if it had to stop early.
#pragma once

#include "swsph_internal.h"

namespace swsph {

constexpr int WORKCAP = 256;            // work queue items (per wavefront)
constexpr int LEAFCAP = 128;            // leaves handed out per batch
constexpr int START_MAX = 64;           // cells of the first search level
constexpr int SEARCH_MAX_CHUNKS = 1 << 14;

struct SearchMem {
    uint64_t work[WORKCAP];
    int32_t lbeg[LEAFCAP];
    int32_t lcnt[LEAFCAP];
    int32_t lshift[LEAFCAP];
};

struct TileGeom {
    float lo[3], hi[3];
};

struct SearchState {
    int head, tail, nleaf, chunks;
};

__device__ __forceinline__ uint64_t pack_item(uint32_t mort, int level, int shift) {
    return (uint64_t)mort | ((uint64_t)level << 32) | ((uint64_t)shift << 40);
}

__device__ __forceinline__ int floor_div(int a, int q) {
    return a >= 0 ? a / q : -((-a + q - 1) / q);
}

// Shift code of a periodic image: (sx+1) + 3 (sy+1) + 9 (sz+1), s in {-1,0,1}.
__device__ __forceinline__ void shift_of(int code, int& sx, int& sy, int& sz) {
    sx = code % 3 - 1;
    sy = (code / 3) % 3 - 1;
    sz = code / 9 - 1;
}

__device__ inline void search_init(SearchMem& m, SearchState& st, const BoxInfo& bi,
                                   const TileGeom& g, float Rstart) {
    const int lane = lane_id();
    const float L = (float)bi.L;
    if (!(Rstart > 0.f)) Rstart = 0.5f * L;
    Rstart = fminf(Rstart, 0.5f * L);
    const int kmax = bi.k < 10 ? bi.k : 10;
    int l = 0;
    while (l < kmax && L / (float)(1 << (l + 1)) >= Rstart) ++l;
    int c0[3], nd[3], total = 1;
    for (int guard = 0; guard < 12; ++guard) {
        const float w = L / (float)(1 << l);
        total = 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float a = floorf((g.lo[d] - Rstart) / w), b = floorf((g.hi[d] + Rstart) / w);
            if (!(a == a)) a = 0.f;   // NaN bounding box: one cell
            if (!(b == b)) b = a;
            c0[d] = (int)a;
            nd[d] = (int)b - (int)a + 1;
            if (nd[d] < 1) nd[d] = 1;
            if (nd[d] > 64) nd[d] = 64;
            total *= nd[d];
        }
        if (total <= START_MAX || l == 0) break;
        --l;
    }
    if (total > START_MAX) total = START_MAX;
    const int q = 1 << l;
    if (lane < total) {
        int e = lane;
        int c[3];
        c[0] = c0[0] + e % nd[0]; e /= nd[0];
        c[1] = c0[1] + e % nd[1]; e /= nd[1];
        c[2] = c0[2] + e;
        int shift = 0, mul = 1;
        uint32_t w3[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int s = floor_div(c[d], q);
            if (s < -1) s = -1;
            if (s > 1) s = 1;
            int wc = c[d] - s * q;
            if (wc < 0) wc = 0;
            if (wc >= q) wc = q - 1;
            w3[d] = (uint32_t)wc;
            shift += (s + 1) * mul;
            mul *= 3;
        }
        m.work[lane] = pack_item(morton3(w3[0], w3[1], w3[2]), l, shift);
    }
    st.head = 0;
    st.tail = total;
    st.nleaf = 0;
    st.chunks = 0;
    wave_sync();
}

// Fill the leaf buffer (at most LEAFCAP) or finish.  Returns true when the
// search is done (queue empty, or the chunk cap was reached).
// CELL_H: a cell also stays while its largest support (times hm) reaches
// the tile.
template <bool CELL_H>
__device__ inline bool search_step(SearchMem& m, SearchState& st, const BoxInfo& bi,
                                   const TileGeom& g, float R2, const int32_t* __restrict__ cstart,
                                   const float* __restrict__ hpyr, float hm, int leaf_max,
                                   Counters* cnt) {
    const int lane = lane_id();
    const float L = (float)bi.L;
    const float pad = 1.0f + 1.0e-4f;
    const int kmax = bi.k < 10 ? bi.k : 10;
    while (st.head < st.tail && st.nleaf + WAVE <= LEAFCAP) {
        if (++st.chunks > SEARCH_MAX_CHUNKS) {
            if (lane == 0) latch(cnt, SWSPH_ST_LOOPCAP);
            st.head = st.tail;
            break;
        }
        const int chunk = min(WAVE, st.tail - st.head);
        const bool has = lane < chunk;
        const uint64_t it = has ? m.work[(st.head + lane) & (WORKCAP - 1)] : 0ull;
        st.head += chunk;
        int decision = 0;  // 0 drop, 1 leaf, 2 refine
        int32_t beg = 0, num = 0;
        const uint32_t mort = (uint32_t)it;
        int level = (int)((it >> 32) & 0xff);
        const int shift = (int)((it >> 40) & 0xff);
        if (level > kmax) level = kmax;
        if (has) {
            const int sh = 3 * (kmax - level);
            const int64_t fb = bi.fine_off + ((int64_t)mort << sh);
            const int64_t fe = fb + ((int64_t)1 << sh);
            beg = cstart[fb];
            num = cstart[fe] - beg;
            if (num > 0) {
                const float w = L / (float)(1 << level);
                int sv[3];
                shift_of(shift, sv[0], sv[1], sv[2]);
                const uint32_t cc[3] = {compact3(mort), compact3(mort >> 1), compact3(mort >> 2)};
                float gap2 = 0.f, far2 = 0.f;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const float a = (float)cc[d] * w + (float)sv[d] * L;
                    const float b = a + w;
                    const float gp = fmaxf(0.f, fmaxf(a - g.hi[d], g.lo[d] - b));
                    const float fr = fmaxf(0.f, fmaxf(g.lo[d] - a, b - g.hi[d]));
                    gap2 += gp * gp;
                    far2 += fr * fr;
                }
                float crit = R2 * pad;
                if (CELL_H) {
                    const float hc = hpyr[bi.pyr_off + pyr_level_off(level) + mort] * hm;
                    crit = fmaxf(crit, hc * hc * pad);
                }
                if (gap2 < crit) {
                    const bool full = far2 < R2;
                    decision = (level < kmax && num > leaf_max && !full) ? 2 : 1;
                }
            }
        }
        unsigned long long rm = ballot(decision == 2);
        int nref = __popcll(rm);
        if (nref > 0 && (st.tail - st.head) + 8 * nref > WORKCAP) {
            if (decision == 2) decision = 1;
            rm = 0;
            nref = 0;
        }
        if (decision == 2) {
            const int pos = st.tail + 8 * mbcnt(rm);
#pragma unroll
            for (int c = 0; c < 8; ++c)
                m.work[(pos + c) & (WORKCAP - 1)] = pack_item(mort * 8u + (uint32_t)c, level + 1, shift);
        }
        st.tail += 8 * nref;
        const unsigned long long lm = ballot(decision == 1);
        if (decision == 1) {
            const int pos = st.nleaf + mbcnt(lm);
            m.lbeg[pos] = beg;
            m.lcnt[pos] = num;
            m.lshift[pos] = shift;
        }
        st.nleaf += __popcll(lm);
        wave_sync();
    }
    return st.head >= st.tail;
}

// Exclusive prefix sum across the wavefront (total in `total`); every lane
// must be active.  Inclusive sums within each row of 16 lanes by DPP row
// shifts (source lanes before the row start read 0), then the row totals
// from lanes 15, 31, 47 and 63 by register reads: no LDS round trip.
template <int CTRL>
__device__ __forceinline__ int row_shr_add(int x) {
    return x + __builtin_amdgcn_update_dpp(0, x, CTRL, 0xf, 0xf, true);
}
__device__ __forceinline__ int wave_excl_scan(int v, int& total) {
    const int lane = lane_id();
    int x = v;
    x = row_shr_add<0x111>(x);  // row_shr:1
    x = row_shr_add<0x112>(x);  // row_shr:2
    x = row_shr_add<0x114>(x);  // row_shr:4
    x = row_shr_add<0x118>(x);  // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(x, 15), r1 = __builtin_amdgcn_readlane(x, 31);
    const int r2 = __builtin_amdgcn_readlane(x, 47), r3 = __builtin_amdgcn_readlane(x, 63);
    const int row = lane >> 4;
    x += (row > 0 ? r0 : 0) + (row > 1 ? r1 : 0) + (row > 2 ? r2 : 0);
    total = r0 + r1 + r2 + r3;
    return x - v;
}

}  // namespace swsph
