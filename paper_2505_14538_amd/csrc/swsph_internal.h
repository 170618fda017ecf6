// swsph_internal.h -- shared definitions of the gfx950 SPH library (device
// helpers, workspace layout, per-box tables).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swsph.h"

// Occupancy target of a kernel (wavefronts per SIMD the register
// allocation must allow).
#ifndef SWSPH_WAVES_PER_EU
#define SWSPH_WAVES_PER_EU(n) __attribute__((amdgpu_waves_per_eu(n)))
#endif
// Dynamic LDS of a kernel.
#ifndef SWSPH_DYN_SHARED
#define SWSPH_DYN_SHARED extern __shared__ __align__(16)
#endif

namespace swsph {

constexpr int WAVE = 64;
constexpr double PI_D = 3.14159265358979323846;

// ------------------------------------------------------------------ tables

// Per-box geometry, computed on the host from the particle counts and box
// sizes and copied into the workspace by swsph_bin.
struct BoxInfo {
    double L;           // side length
    int64_t start;      // first particle of the box in binned (sorted) order
    int64_t count;      // particles in the box
    int64_t fine_off;   // offset of the box's cells in the fine cell table
    int64_t pyr_off;    // offset of the box's level-0 entry in the H-max pyramid
    int32_t k;          // fine level: 2^k cells per dimension
    int32_t pad[3];
};

// One i-tile task: the particles of one cubic cell of the box's cell tree
// (the coarsest cell holding at most `tile` particles), or a run of at most
// `tile` particles of an overfull finest cell.  Consecutive binned particles.
struct Tile {
    int32_t begin;      // first binned particle
    int32_t count;      // particles (1 .. tile size)
    int32_t box;
    int32_t flags;
    float lo[3], hi[3]; // bounding box of the tile's particles
    float hmax;         // largest smoothing length in the tile
    float cost;         // work estimate (candidate pairs)
};

// Device counters (start of the workspace).  All 64-bit for atomics.
struct Counters {
    unsigned long long status;
    unsigned long long pairs_tested[4];
    unsigned long long pairs_inside[4];
    unsigned long long newton_sweeps;
    unsigned long long newton_max;
    unsigned long long newton_failed;
    unsigned long long listed;
    unsigned long long restages;
    unsigned long long queue[4][8];    // task-queue heads per loop (8: one per XCD segment)
    unsigned long long build_queue[8]; // item-queue heads of the task builds
    unsigned long long n_tiles;        // tiles of the gradient/force (and adjoint) loops
    unsigned long long n_tiles_d;      // tiles of the density loop
    unsigned long long n_fix;          // tiles listed for the current density fix-up pass
    unsigned long long cand_used;      // task-list entries taken by the current build
    unsigned long long dens_listed;    // density tiles that swept per-particle neighbour lists
    unsigned long long n_items;        // single-launch step: density plus gradient/force tiles
    unsigned long long single_redo;    // single-launch step: gradient/force tiles redone after it
    unsigned long long reserved[3];
};

enum Loop { LOOP_DENSITY = 0, LOOP_GRADIENT = 1, LOOP_FORCE = 2, LOOP_BACKWARD = 3 };

// Byte offsets of every workspace region (computed on the host).
struct Layout {
    uint64_t counters, boxtab;
    uint64_t keys, slot, tmpidx, perm, rank;  // slot/tmpidx: reused for the tile scan
    uint64_t fine_count, cstart, scan_part;
    uint64_t pos4, vel4, hs, dens4, hmaxpyr;
    uint64_t tiles, order, tiles_d, order_d, dparent, ord_table, ord_base;
    // task lists (candidate entries per tile) and density fix-up state
    uint64_t cand_cnt, cand_off, cands, trad, tflag, fbox;
    // single-launch step: density fix-up radii, gradient/force tiles to
    // redo, the launch's task order, per-box phase words and tile totals
    uint64_t trad_d, fredo, forder, boxph;
    // sorted-order results
    uint64_t d_out;     // 10 arrays of T: h rho rho_dh wcount wcount_dh div cx cy cz f
    uint64_t d_int;     // 2 arrays of int32: nngb iters
    uint64_t g_out;     // 3 arrays of T (the third: alpha_V,ngb of the switch loops)
    uint64_t f_out;     // 4 arrays of T
    uint64_t f_int;     // 1 array of int32
    uint64_t adj;       // adjoint scratch: 16 arrays of T
    uint64_t total;
};

// ----------------------------------------------------------- device helpers

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using V4 = typename Vec4<T>::type;

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot((int)p); }

// Lanes below this one whose bit is set in mask.
__device__ __forceinline__ int mbcnt(unsigned long long mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Make LDS stores of every lane visible to every lane of the same wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// XCD (accelerator complex die) the wavefront runs on: the hardware XCC_ID
// register (read only).
__device__ __forceinline__ int xcc_id() {
    return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15;  // hwreg(XCC_ID, 0, 4)
}

// Items [0, n) handed to wavefronts on demand, so a few costly items do not
// hold up a static schedule.  With `split` the range is cut into NSEG
// segments (one per XCD; heads[NSEG] start at zero) and a wavefront pops
// from its own XCD's segment first (hardware XCC id), then helps the others;
// otherwise heads[0] serves the whole range.  One item per pop, the next pop
// issued before the current item runs (its latency hides behind the work).
// f(k) is called by the whole wavefront at one site.  Bounded: every
// iteration takes one item or moves to the next segment.
constexpr int NSEG = 8;

// A pop that is not prefetched (a wavefront's first on a segment): `step`
// more positions of the counter, or `limit` (the segment's length: drained)
// without an atomic when a plain read already shows the counter there.  The
// counter only grows, so that read cannot report a drained segment early; a
// drained queue then costs each wavefront a load instead of a
// read-modify-write on one shared address (thousands of those serialise: an
// empty launch took tens of microseconds).  Lane 0 only.
__device__ __forceinline__ int queue_pop_checked(unsigned long long* head, unsigned long long step,
                                                 int64_t limit) {
    const unsigned long long cur =
        __hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((int64_t)cur >= limit) return (int)limit;
    return (int)atomicAdd(head, step);
}
template <class F>
__device__ __forceinline__ void for_each_item(unsigned long long* heads, int64_t n, bool split,
                                              F&& f) {
    const int nseg = split ? NSEG : 1;
    const int x0 = split ? xcc_id() % NSEG : 0;
    int y = 0, x = x0;
    int64_t b = split ? n * x / NSEG : 0, e = split ? n * (x + 1) / NSEG : n;
    int v = 0;
    if (lane_id() == 0) v = queue_pop_checked(&heads[x], 1ull, e - b);
    int64_t k = b + (int64_t)uniform(v);
    const int64_t guard_max = n + 2 * NSEG + 2;
    for (int64_t guard = 0; guard < guard_max; ++guard) {
        if (k >= e) {
            if (++y >= nseg) break;
            x = (x0 + y) % NSEG;
            b = n * x / NSEG;
            e = n * (x + 1) / NSEG;
            int w = 0;
            if (lane_id() == 0) w = queue_pop_checked(&heads[x], 1ull, e - b);
            k = b + (int64_t)uniform(w);
            continue;
        }
        int vn = 0;
        if (lane_id() == 0) vn = (int)atomicAdd(&heads[x], 1ull);
        f(k);
        k = b + (int64_t)uniform(vn);
    }
}

// The value lane c holds (c the same in every lane): a register read across
// lanes, no LDS round trip.
__device__ __forceinline__ int lane_val(int v, int c) { return __builtin_amdgcn_readlane(v, c); }
__device__ __forceinline__ float lane_val(float v, int c) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), c));
}
__device__ __forceinline__ double lane_val(double v, int c) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, c);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), c);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ float shfl_xor(float v, int m) { return __shfl_xor(v, m, WAVE); }
__device__ __forceinline__ double shfl_xor(double v, int m) { return __shfl_xor(v, m, WAVE); }
__device__ __forceinline__ int shfl_xor(int v, int m) { return __shfl_xor(v, m, WAVE); }

template <typename T> __device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) { T o = shfl_xor(v, m); v = o > v ? o : v; }
    return v;
}
template <typename T> __device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) { T o = shfl_xor(v, m); v = o < v ? o : v; }
    return v;
}
__device__ __forceinline__ unsigned long long shfl_xor(unsigned long long v, int m) {
    return __shfl_xor(v, m, WAVE);
}
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
    return v;
}

// Squared distance in a fixed, unfused order: ((dx*dx + dy*dy) + dz*dz).
// Integer neighbour counts depend on it bit for bit, so no product may be
// contracted into an addition here.
__device__ __forceinline__ float dist2_unfused(float dx, float dy, float dz) {
#pragma clang fp contract(off)
    float a = dx * dx;
    float b = dy * dy;
    float c = dz * dz;
    float s = a + b;
    return s + c;
}
__device__ __forceinline__ double dist2_unfused(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    double a = dx * dx;
    double b = dy * dy;
    double c = dz * dz;
    double s = a + b;
    return s + c;
}
__device__ __forceinline__ float sub_unfused(float a, float b) { return a - b; }
__device__ __forceinline__ float add_unfused(float a, float b) { return a + b; }
__device__ __forceinline__ float mul_unfused(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double mul_unfused(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}

// A coordinate as a float bound: rounded down (up) when the value is a
// double that float does not hold exactly, so a box stays around its points.
__device__ __forceinline__ float float_down(float v) { return v; }
__device__ __forceinline__ float float_up(float v) { return v; }
__device__ __forceinline__ float float_down(double v) {
    const float f = (float)v;
    return (double)f > v ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float float_up(double v) {
    const float f = (float)v;
    return (double)f < v ? nextafterf(f, INFINITY) : f;
}

__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double fast_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

__device__ __forceinline__ void latch(Counters* c, unsigned bits) {
    atomicOr(&c->status, (unsigned long long)bits);
}

// Morton code: bit b of cx -> bit 3b, of cy -> 3b+1, of cz -> 3b+2.
__host__ __device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}
__host__ __device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030C30C3u;
    v = (v | (v >> 4)) & 0x0300F00Fu;
    v = (v | (v >> 8)) & 0x030000FFu;
    v = (v | (v >> 16)) & 0x000003FFu;
    return v;
}

// Element stride of the adjoint's per-particle scratch arrays: n rounded up
// to a multiple of 4, so every array (and the 4-vector views over four of
// them) starts 4-element aligned inside the 256-byte aligned region.
__host__ __device__ __forceinline__ int64_t adj_stride(int64_t n) { return (n + 3) & ~int64_t(3); }

// Offset of level l inside one box's pyramid (levels 0..k, 8^l cells each).
__host__ __device__ __forceinline__ int64_t pyr_level_off(int l) {
    return ((int64_t(1) << (3 * l)) - 1) / 7;
}

// Box of a cell key: the last box whose fine-cell range starts at or
// before it (every box owns at least one fine cell, so the offsets rise
// strictly).  Keys come from the cell table itself, so this never disagrees
// with the binned layout, whatever per-box counts the caller declared.
__device__ __forceinline__ int box_of_key(uint32_t key, int32_t n_box,
                                          const BoxInfo* __restrict__ boxtab) {
    int lo = 0, hi = n_box - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (boxtab[mid].fine_off <= (int64_t)key) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace swsph
