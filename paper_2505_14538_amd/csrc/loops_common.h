// loops_common.h -- shared pieces of the loop kernels (forward and adjoint):
// per-wavefront LDS layout, kernel arguments, the staging of a tile's
// j-particles from its task list, and M4 kernel pieces.
#pragma once

#include <type_traits>

#include "launch.h"
#include "search.h"

namespace swsph {

constexpr int WPB = 4;  // wavefronts per workgroup
constexpr int LC = 32;  // entries of a lane's hit list

template <typename T, int CAP, int NV>
struct WaveMem {
    // hit-list length: 16 for the loops staging four or more 4-vectors per
    // particle, so the gradient/force kernel's 128 staged particles and
    // lists take 10 KB per wavefront and four wavefronts per SIMD fit LDS
    static constexpr int HL = NV >= 4 ? 16 : LC;
    static constexpr int NENT = HL * WAVE;
    V4<T> s[NV][CAP];          // staged j-particles
    union {
        uint16_t lst[HL][WAVE];  // per-lane hit lists (staged indices), column per lane
        uint16_t ent[NENT];      // density: per-i neighbour lists (staged indices)
    };
};

template <typename T>
struct KArgs {
    const BoxInfo* boxtab;
    const Tile* tiles;
    const int32_t* order;      // task list: tile indices in queue order
    const unsigned long long* ntask;  // its length (device)
    int64_t tile_cap;          // bound of the device tile count (cnt->n_tiles)
    int32_t task;              // per-task launch: the task to run
    const int32_t* cand_cnt;
    const int32_t* cand_off;
    const uint32_t* cands;
    int64_t cand_cap;
    float* trad;
    int32_t* tflag;
    float* fbox;               // density fix-ups: box of each flagged tile's pending particles
    const V4<T>* pos4;
    const V4<T>* vel4;
    T* hs;
    const V4<T>* dens4;
    const V4<T>* aux4;         // adjoint passes: per-particle staging data
    T* out;                    // sorted outputs, arrays of n
    T* gout;                   // joint gradient/force loop: the gradient outputs
    const int32_t* parent;     // density first pass: each tile's list is its parent's (or null)
    T dmargin;                 // density: staged radius over the largest guessed support
    int32_t* iout;             // sorted int outputs, arrays of n
    int64_t n;
    Counters* cnt;
    unsigned long long* queue;        // NXCD queue heads
    int32_t xcd_split;                // queue: one Morton segment of the task list per XCD
    T eta, eps, gamma, alpha, beta, h_tol;
    int32_t h_max_iter;
    uint32_t flags;
    int32_t fixup;             // density: 0 first pass, 1 fix-up pass, 2 last fix-up pass
    // single-launch step (null otherwise): density tiles also write
    // (rho, f, c, A) per particle and report to their box's phase word
    // (checking h against the guesses hguess); gradient/force tiles wait for
    // it and flag themselves for a redo
    V4<T>* dens4_out;
    const T* hguess;
    uint32_t* boxph;           // per box: done count | BOX_REDO (one cache line each);
                               // then its density tiles; then its smallest
                               // gradient/force list radius (float bits)
    int32_t* fredo;
    int32_t n_box;
    int32_t qchunk;            // queue: tasks per pop
};

constexpr int QCHUNK = 2;  // tasks per queue pop (the loops' default)

// Box phase words sit one cache line apart (their atomics and polls do not
// share lines); the per-box totals and radii follow them.
constexpr int BOX_STRIDE = 32;

// Phase word of a box in the single-launch step: density tiles done (low
// bits) and the redo bit (some h of the box ended beyond the margin its
// gradient/force lists were built with, or a tile needs a wider search).
constexpr uint32_t BOX_REDO = 1u << 31;
constexpr uint32_t BOX_DONE = BOX_REDO - 1u;

// Lane mapping of a tile of c particles (c <= 64): c i-slots times S =
// floor(64 / c) streams, lane = i-slot + c * stream; the 64 - S c lanes
// left over are unused (their tests are off).  Each stream of an i-particle
// walks every S-th staged j-particle.
struct LaneMap {
    int T_i, S, li, js;
    __device__ __forceinline__ bool used() const { return js < S; }
};
__device__ __forceinline__ LaneMap lane_map(int c) {
    LaneMap q;
    q.T_i = c < 1 ? 1 : (c > WAVE ? WAVE : c);
    q.S = WAVE / q.T_i;
    const int lane = lane_id();
    q.js = lane / q.T_i;
    q.li = lane - q.js * q.T_i;
    return q;
}

// Sum (max) over the streams of each i-slot, returned in every lane of the
// slot: a tree over stream indices with lane permutes (fixed order, so the
// result is deterministic), then a broadcast from the slot's stream 0.
template <typename V> __device__ __forceinline__ V stream_sum(V v, const LaneMap& q) {
    const int lane = lane_id();
    for (int m = 1; m < q.S; m <<= 1) {
        const int src = q.li + q.T_i * (q.js + m);
        const V o = __shfl(v, src < WAVE ? src : lane, WAVE);
        if ((q.js & (2 * m - 1)) == 0 && q.js + m < q.S) v += o;
    }
    return __shfl(v, q.li, WAVE);
}
template <typename V> __device__ __forceinline__ V stream_max(V v, const LaneMap& q) {
    const int lane = lane_id();
    for (int m = 1; m < q.S; m <<= 1) {
        const int src = q.li + q.T_i * (q.js + m);
        const V o = __shfl(v, src < WAVE ? src : lane, WAVE);
        if ((q.js & (2 * m - 1)) == 0 && q.js + m < q.S && o > v) v = o;
    }
    return __shfl(v, q.li, WAVE);
}

// Pair loop over the staged j-particles with per-lane compaction.  Lane
// (i-slot, stream js) runs the distance test over the staged indices
// js, js + S, ...; the hits go, in index order, to the lane's own list in
// LDS, and whenever some list could overflow (and at the end) every lane
// runs the pair body over its list with the wavefront in step.  The body
// thus runs with nearly all lanes busy instead of under the divergence of
// the test (only a few of the tested pairs lie inside the support), and
// each lane still accumulates its pairs in staged order, so results do not
// depend on the list length.  Tests go PL_U at a time, the body two at a
// time (the second pair's reads overlap the first's arithmetic); loop
// control is wavefront-uniform.  test(k, ok) must return false when !ok (k
// is then a valid but repeated index).
constexpr int PL_U = 4;

template <class WM, class Test, class Body>
__device__ __forceinline__ void pair_loop(WM& m, int ns, int js, int S, Test&& test,
                                          Body&& body) {
    const int lane = lane_id();
    ns = uniform(ns);
    S = uniform(S);
    int c = 0;
    auto drain = [&]() {
        for (int e = 0; ballot(e < c) != 0ull; e += 2) {
            const int k0 = e < c ? (int)m.lst[e][lane] : -1;
            const int k1 = e + 1 < c ? (int)m.lst[e + 1][lane] : -1;
            if (k0 >= 0) body(k0);
            if (k1 >= 0) body(k1);
        }
        c = 0;
    };
    const int step = S * PL_U;
    // one group of PL_U tests per lane; a full group (k0 + step <= ns) needs
    // no bounds checks, only the last one does
    auto group = [&](int k0, auto full) {
        bool hit[PL_U];
#pragma unroll
        for (int u = 0; u < PL_U; ++u) {
            const int k = k0 + js + u * S;
            if constexpr (decltype(full)::value) hit[u] = test(k, true);
            else hit[u] = test(k < ns ? k : ns - 1, k < ns);
        }
        // appended without a branch: every index is written at slot c and
        // kept by advancing c on a hit.  A list holds at most HL - PL_U
        // entries when a group starts (drained otherwise), so every write
        // stays below HL; a slot at or past c is never read.
#pragma unroll
        for (int u = 0; u < PL_U; ++u) {
            m.lst[c][lane] = (uint16_t)(k0 + js + u * S);
            c += hit[u] ? 1 : 0;
        }
        if (ballot(c > WM::HL - PL_U) != 0ull) drain();
    };
    int k0 = 0;
    for (; k0 + step <= ns; k0 += step) group(k0, std::true_type{});
    if (k0 < ns) group(k0, std::false_type{});
    drain();
}

// Keep, in order and in place, the staged j-particles (one 4-vector each,
// the density loop's layout) whose distance to the tile box is below
// sqrt(R2) (staged positions already carry their periodic image).  Writes
// never pass the chunk being read, so in place is safe.  Returns the new
// count.
template <typename T, int CAP>
__device__ int compact_staged(WaveMem<T, CAP, 1>& m, int ns, const TileGeom& g, T R2) {
    const int lane = lane_id();
    int out = 0;
    for (int b = 0; b < ns; b += WAVE) {
        const int k = b + lane;
        const bool have = k < ns;
        V4<T> s0{};
        bool keep = false;
        if (have) {
            s0 = m.s[0][k];
            const T x = s0.x, y = s0.y, z = s0.z;
            const T gx = max((T)0, max((T)g.lo[0] - x, x - (T)g.hi[0]));
            const T gy = max((T)0, max((T)g.lo[1] - y, y - (T)g.hi[1]));
            const T gz = max((T)0, max((T)g.lo[2] - z, z - (T)g.hi[2]));
            keep = dist2_unfused(gx, gy, gz) < R2;
        }
        const unsigned long long km = ballot(keep);
        wave_sync();
        if (keep) m.s[0][out + mbcnt(km)] = s0;
        out += __popcll(km);
        wave_sync();
    }
    return out;
}

// Sums over aligned groups of S contiguous lanes (S a power of two, the
// same in every lane), returned in every lane of the group: butterflies on
// DPP lane permutes within rows of 16 (quad swaps, half-row and row
// mirrors), a swizzle across the two rows of each half-wavefront, and for
// S = 64 the two halves read from lanes 0 and 32.  Floating-point addition
// is commutative, so every lane of a group gets the same bits.
template <int CTRL> __device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL> __device__ __forceinline__ float dpp_v(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double dpp_v(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = dpp_i<CTRL>((int)(unsigned)b), hi = dpp_i<CTRL>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL> __device__ __forceinline__ int dpp_v(int v) { return dpp_i<CTRL>(v); }
constexpr int SWZ_XOR16 = 0x1f | (0x10 << 10);  // ds_swizzle bit mode: lane ^ 16 within 32
__device__ __forceinline__ int swz16(int v) { return __builtin_amdgcn_ds_swizzle(v, SWZ_XOR16); }
__device__ __forceinline__ float swz16(float v) { return __int_as_float(swz16(__float_as_int(v))); }
__device__ __forceinline__ double swz16(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = swz16((int)(unsigned)b), hi = swz16((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <typename V> __device__ __forceinline__ V group_sum(V v, int S) {
    if (S >= 2) v += dpp_v<0xb1>(v);   // quad_perm 1,0,3,2: lane ^ 1
    if (S >= 4) v += dpp_v<0x4e>(v);   // quad_perm 2,3,0,1: lane ^ 2
    if (S >= 8) v += dpp_v<0x141>(v);  // row_half_mirror: the other quad of 8
    if (S >= 16) v += dpp_v<0x140>(v); // row_mirror: the other 8 of the row
    if (S >= 32) v += swz16(v);        // the other row of 32
    if (S >= 64) v = lane_val(v, 0) + lane_val(v, 32);
    return v;
}

// Lane mapping of the density loop: a tile of c particles (c <= 64) gets
// c i-slots of S = the largest power of two <= 64 / c streams each, the
// streams of a slot on contiguous lanes (lane = S i-slot + stream), so
// sums over a slot's streams are group_sum(., S).
struct GroupMap {
    int c, S, li, js;
    bool act;
};
__device__ __forceinline__ GroupMap group_map(int c) {
    GroupMap q;
    q.c = c < 1 ? 1 : (c > WAVE ? WAVE : c);
    int S = 1;
    while (2 * S * q.c <= WAVE) S *= 2;
    q.S = S;
    const int lane = lane_id();
    q.act = lane < q.c * S;
    q.li = q.act ? lane / S : 0;
    q.js = lane - (lane / S) * S;
    return q;
}

// loop kinds: forward loops, the three pair passes of the adjoint, and the
// gradient and force loops with time-dependent switches (1 is unused: the
// gradient loop of the plain scheme runs inside the force loop kernel)
enum { L_DENS = 0, L_FORCE = 2, L_ADJA = 3, L_ADJC = 4, L_ADJD = 5, L_GSW = 6, L_FSW = 7 };

template <int LK> struct LoopNV;
template <> struct LoopNV<L_DENS> { static constexpr int NV = 1; };
template <> struct LoopNV<L_FORCE> { static constexpr int NV = 4; };
template <> struct LoopNV<L_ADJA> { static constexpr int NV = 5; };
template <> struct LoopNV<L_ADJC> { static constexpr int NV = 2; };
template <> struct LoopNV<L_ADJD> { static constexpr int NV = 2; };
template <> struct LoopNV<L_GSW> { static constexpr int NV = 3; };
template <> struct LoopNV<L_FSW> { static constexpr int NV = 5; };

// cull with the symmetric criterion r < max(H_i, H_j)?
template <int LK> struct Symmetric {
    static constexpr bool value = LK == L_FORCE || LK == L_ADJA || LK == L_ADJC ||
                                  LK == L_ADJD || LK == L_FSW;
};

template <typename T> __device__ __forceinline__ T int_as(int32_t v);
template <> __device__ __forceinline__ float int_as<float>(int32_t v) { return __int_as_float(v); }
template <> __device__ __forceinline__ double int_as<double>(int32_t v) { return (double)v; }
template <typename T> __device__ __forceinline__ int32_t as_int(T v);
template <> __device__ __forceinline__ int32_t as_int<float>(float v) { return __float_as_int(v); }
template <> __device__ __forceinline__ int32_t as_int<double>(double v) { return (int32_t)v; }

// The j-data a loop stages, gathered for one candidate in one go.
template <int LK, typename T> struct JData {
    V4<T> p, v, d, x;  // pos4 (x, y, z, m), vel4, dens4 (rho, f, c, A), aux4 (adjoint)
    T h;
};
template <int LK, typename T>
__device__ __forceinline__ void gather_j(const KArgs<T>& a, int j, JData<LK, T>& r) {
    r.p = a.pos4[j];
    constexpr bool VD = LK == L_FORCE || LK == L_ADJA || LK == L_GSW || LK == L_FSW;
    constexpr bool X = LK == L_ADJA || LK == L_ADJC || LK == L_ADJD || LK == L_GSW || LK == L_FSW;
    if (VD) r.v = a.vel4[j];
    if (VD) r.d = a.dens4[j];
    if (X) r.x = a.aux4[j];
    if (Symmetric<LK>::value) r.h = a.hs[j];
}

// Stream the candidate list of tile lt (the tile's own, or for a density
// tile in its first pass the list of the gradient/force tile containing it)
// through the lanes and stage it in LDS.
// Per batch of 64 candidates the entries (read one batch ahead) give the
// j-particles, and every field the loop needs is gathered at once, so a
// batch costs one memory round trip.  The cull here (radius R from the
// tile box; for the symmetric loops also the j-particle's own support)
// keeps the candidates the tile needs: all of its own list unless the caller
// passes a smaller R, a part of a parent's list.  flush(CAP) is called when
// the buffer is full and more survivors arrive (the buffer is empty
// afterwards), so a list and any longer list holding the same survivors in
// the same order stage and flush identically.  Returns the number of staged
// survivors left for the caller.
template <int LK, typename T, int CAP, class WM, class Flush>
__device__ int stage_tile(WM& m, const KArgs<T>& a, int lt, const BoxInfo& bi, const TileGeom& g,
                          T R2, int& flushes, Flush&& flush) {
    const int lane = lane_id();
    const int64_t off = uniform(a.cand_off[lt]);
    int64_t nc = uniform(a.cand_cnt[lt]);
    if (off < 0) nc = 0;
    if (off + nc > a.cand_cap) nc = a.cand_cap > off ? a.cand_cap - off : 0;
    const T L = (T)bi.L;
    int nsurv = 0;
    flushes = 0;
    uint32_t e_next = lane < nc ? a.cands[off + lane] : 0u;
    for (int64_t base = 0; base < nc; base += WAVE) {
        const bool have = base + lane < nc;
        const uint32_t e = e_next;
        int j = (int)(e & 0x3ffffffu);
        if (j >= a.n) j = 0;  // cannot happen with a valid list
        JData<LK, T> r;
        if (have) gather_j<LK, T>(a, j, r);
        if (base + WAVE + lane < nc) e_next = a.cands[off + base + WAVE + lane];
        bool pass = false;
        T xs = 0, ys = 0, zs = 0;
        if (have) {
            int sx, sy, sz;
            shift_of((int)(e >> 26), sx, sy, sz);
            xs = r.p.x + (T)sx * L;
            ys = r.p.y + (T)sy * L;
            zs = r.p.z + (T)sz * L;
            const T gx = max((T)0, max((T)g.lo[0] - xs, xs - (T)g.hi[0]));
            const T gy = max((T)0, max((T)g.lo[1] - ys, ys - (T)g.hi[1]));
            const T gz = max((T)0, max((T)g.lo[2] - zs, zs - (T)g.hi[2]));
            const T d2 = dist2_unfused(gx, gy, gz);
            T crit = R2;
            if (Symmetric<LK>::value) {
                const T Hj = mul_unfused(a.eps, r.h);
                crit = max(crit, mul_unfused(Hj, Hj));
            }
            pass = d2 < crit;
        }
        // the staged record of this lane's candidate (the loop's layout)
        V4<T> q0{}, q1{}, q2{}, q3{}, q4{};
        if (pass) {
            const V4<T> pa = r.p, va = r.v;
            if (LK == L_DENS) {
                // image position and the binned index (mass and velocity
                // are read from global memory for the pairs inside)
                q0 = V4<T>{xs, ys, zs, int_as<T>(j)};
            } else if (LK == L_FORCE) {
                // per candidate, not per pair: 1/H_j and the kernel
                // gradient's normalisation 8/(pi H_j^4), reciprocals (the
                // hardware's in FP32) instead of divisions
                const V4<T> da = r.d;
                const T Hj = mul_unfused(a.eps, r.h);
                const T ihj = fast_rcp(Hj);
                const T ih2 = ihj * ihj;
                q0 = V4<T>{xs, ys, zs, mul_unfused(Hj, Hj)};
                q1 = V4<T>{va.x, va.y, va.z, da.z};
                q2 = V4<T>{pa.w, pa.w * da.w, pa.w * da.y, ihj};
                q3 = V4<T>{da.x, (T)(8.0 / PI_D) * ih2 * ih2, va.w, pa.w * fast_rcp(da.x)};
            } else if (LK == L_GSW) {
                // gradient loop with switches: (m_j / rho_j), c_j, u_j and
                // alpha_V,j (aux4 = alpha_V, B, alpha_c, 0)
                const V4<T> da = r.d;
                q0 = V4<T>{xs, ys, zs, pa.w / da.x};
                q1 = V4<T>{va.x, va.y, va.z, da.z};
                q2 = V4<T>{va.w, r.x.x, (T)0, (T)0};
            } else if (LK == L_FSW) {
                // force loop with switches: the plain force record plus the
                // pressure and the switch values of j
                const V4<T> da = r.d;
                const T Hj = mul_unfused(a.eps, r.h);
                q0 = V4<T>{xs, ys, zs, mul_unfused(Hj, Hj)};
                q1 = V4<T>{va.x, va.y, va.z, da.z};
                q2 = V4<T>{pa.w, pa.w * da.w, pa.w * da.y, (T)1 / Hj};
                q3 = V4<T>{da.x, (a.gamma - (T)1) * da.x * va.w, va.w, (T)0};
                q4 = r.x;
            } else if (LK == L_ADJA) {
                const V4<T> da = r.d;   // (rho, f, c, A)
                const V4<T> wj = r.x;   // (dL/dax, dL/day, dL/daz, dL/ddu)
                const T Hj = mul_unfused(a.eps, r.h);
                q0 = V4<T>{xs, ys, zs, mul_unfused(Hj, Hj)};
                q1 = V4<T>{va.x, va.y, va.z, da.z};
                q2 = V4<T>{pa.w, da.w, da.y, (T)1 / Hj};
                q3 = V4<T>{da.x, wj.x, wj.y, wj.z};
                q4 = V4<T>{wj.w, int_as<T>(j), (T)0, (T)0};
            } else {
                // density adjoint: (m, rho_bar, rho'_bar, 1/H); implicit h: (lambda h^3, 1/H, idx, 0)
                const T Hj = mul_unfused(a.eps, r.h);
                q0 = V4<T>{xs, ys, zs, mul_unfused(Hj, Hj)};
                q1 = r.x;
            }
        }
        auto put = [&](int k) {
            constexpr int NV = LoopNV<LK>::NV;
            m.s[0][k] = q0;
            if (NV > 1) m.s[1][k] = q1;
            if (NV > 2) m.s[2][k] = q2;
            if (NV > 3) m.s[3][k] = q3;
            if (NV > 4) m.s[4][k] = q4;
        };
        // survivors fill the buffer in list order; only when it is full and
        // more arrive does it go to flush, so where flushes fall depends on
        // the survivors alone, not on how the list is cut into batches
        const unsigned long long pm = ballot(pass);
        const int cnt = __popcll(pm);
        const int rank = mbcnt(pm);
        const int room = CAP - nsurv;
        if (pass && rank < room) put(nsurv + rank);
        if (cnt > room) {
            wave_sync();
            flush(CAP);
            ++flushes;
            wave_sync();
            if (pass && rank >= room) put(rank - room);
            nsurv = cnt - room;
        } else {
            nsurv += cnt;
        }
        wave_sync();
    }
    return nsurv;
}

// ---------------------------------------------------------------- kernels
// M4 pieces on q = r/H:  w, s1 = 3w + q w', g = w'/q  (all finite at q = 0).

template <typename T>
__device__ __forceinline__ void m4_terms(T q, T inv_q, T& w, T& s1, T& g) {
    // both pieces, then a select: no divergent branch in the pair body
    const T t = (T)1 - q;
    const T q2 = q * q;
    const T t2 = t * t;
    const bool in = q < (T)0.5;
    const T wi = (T)1 + q2 * ((T)6 * q - (T)6), wo = (T)2 * t2 * t;
    const T si = (T)3 + q2 * ((T)36 * q - (T)30), so = (T)6 * t2 * ((T)1 - (T)2 * q);
    const T gi = (T)18 * q - (T)12, go = (T)-6 * t2 * inv_q;
    w = in ? wi : wo;
    s1 = in ? si : so;
    g = in ? gi : go;
}
// q^2 w''(q): with q w'(q) it gives the second derivative of sum_j w(q_j)
// over log h (q scales as 1/h)
template <typename T> __device__ __forceinline__ T m4_q2w2(T q) {
    const T q2 = q * q;
    const T a = q2 * ((T)36 * q - (T)12), b = (T)12 * q2 * ((T)1 - q);
    return q < (T)0.5 ? a : b;
}
// w'(q)
// The larger of two squared radii (b >= 0, a >= 0 or a = -1 for an unused
// lane; neither NaN).  FP32: as integers, since the bit patterns of
// non-negative floats order as the floats do and a negative a loses to any b
// (no NaN quieting, which the float max needs).
__device__ __forceinline__ float max_sq(float a, float b) {
    return __int_as_float(max(__float_as_int(a), __float_as_int(b)));
}
__device__ __forceinline__ double max_sq(double a, double b) { return a > b ? a : b; }

template <typename T> __device__ __forceinline__ T m4_dw(T q) {
    const T t = (T)1 - q;
    const T a = q * ((T)18 * q - (T)12), b = (T)-6 * t * t;
    return q < (T)0.5 ? a : b;
}

__device__ __forceinline__ TileGeom geom_of(const Tile& tl) {
    TileGeom g;
#pragma unroll
    for (int d = 0; d < 3; ++d) { g.lo[d] = tl.lo[d]; g.hi[d] = tl.hi[d]; }
    return g;
}


template <typename T>
inline KArgs<T> make_args(const BinPtrs& b, const Scheme& sc) {
    KArgs<T> a;
    a.boxtab = b.boxtab;
    a.tiles = b.tiles;
    a.order = b.order;
    a.ntask = b.ntiles;
    a.tile_cap = b.tile_cap;
    a.task = 0;
    a.cand_cnt = b.cand_cnt;
    a.cand_off = b.cand_off;
    a.cands = b.cands;
    a.cand_cap = b.cand_cap;
    a.trad = b.trad;
    a.tflag = b.tflag;
    a.fbox = b.fbox;
    a.pos4 = (const V4<T>*)b.pos4;
    a.vel4 = (const V4<T>*)b.vel4;
    a.hs = (T*)b.hs;
    a.dens4 = (const V4<T>*)b.dens4;
    a.aux4 = nullptr;
    a.out = nullptr;
    a.gout = nullptr;
    a.parent = nullptr;
    a.dmargin = (T)((sc.flags & SWSPH_FIXED_H) ? 1.0 : DENS_MARGIN);
    a.iout = nullptr;
    a.n = b.n;
    a.cnt = b.cnt;
    a.queue = nullptr;
    a.xcd_split = sc.order == 1;
    a.eta = (T)sc.eta;
    a.eps = (T)sc.eps;
    a.gamma = (T)sc.gamma;
    a.alpha = (T)sc.alpha;
    a.beta = (T)sc.beta;
    a.h_tol = (T)sc.h_tol;
    a.h_max_iter = sc.h_max_iter;
    a.flags = sc.flags;
    a.fixup = 0;
    a.dens4_out = nullptr;
    a.hguess = nullptr;
    a.boxph = nullptr;
    a.fredo = nullptr;
    a.n_box = b.n_box;
    a.qchunk = QCHUNK;
    return a;
}

// Statistics a wavefront gathers over its tiles (uniform values; added to
// the device counters once per wavefront at the end of a launch, not per
// tile, so hundreds of thousands of small tiles do not queue on a few
// atomic counters).
struct WaveStats {
    unsigned long long tested = 0, inside = 0, sweeps = 0, smax = 0, failed = 0, restages = 0;
    unsigned long long inside_g = 0;  // gradient pairs of the joint gradient/force loop
    unsigned long long listed = 0;    // density tiles swept over neighbour lists
    // per-lane parts (density loop), reduced over the wavefront at the flush
    unsigned long long lane_tested = 0, lane_inside = 0;
    int lane_smax = 0;
    // loop: index of the statistics (LOOP_*); joint: the joint gradient/force
    // kernel, whose tests serve both loops
    __device__ void flush(Counters* c, int loop, bool joint) const {
        // every lane: the wavefront reductions of the per-lane parts
        const unsigned long long lt = wave_sum(lane_tested), li = wave_sum(lane_inside);
        const unsigned long long sm = (unsigned long long)max(smax, (unsigned long long)wave_max(lane_smax));
        if (lane_id() != 0) return;
        if (tested + lt) atomicAdd(&c->pairs_tested[loop], tested + lt);
        if (inside + li) atomicAdd(&c->pairs_inside[loop], inside + li);
        if (joint) {
            if (tested) atomicAdd(&c->pairs_tested[LOOP_GRADIENT], tested);
            if (inside_g) atomicAdd(&c->pairs_inside[LOOP_GRADIENT], inside_g);
        }
        if (sweeps) atomicAdd(&c->newton_sweeps, sweeps);
        if (sm) atomicMax(&c->newton_max, sm);
        if (failed) atomicAdd(&c->newton_failed, failed);
        if (restages) atomicAdd(&c->restages, restages);
        if (listed) atomicAdd(&c->dens_listed, listed);
    }
};

// Task dispatch inside a loop kernel.
//  * queue: every wavefront pops qchunk consecutive tasks at a time until the
//    list is drained (at most tile_cap + 1 pops per list).  With xcd_split
//    the list (in Morton order) is cut into NXCD contiguous segments and a
//    wavefront starts on the segment of the XCD it runs on (hardware XCC
//    id), so each XCD's L2 cache sees a compact region of the box; a
//    wavefront whose segment is drained helps the next ones.
//  * flat: the static round-robin schedule.
//  * per-task: the one task of the launch.
constexpr int NXCD = 8;

// One call site of `run` (the tile body is inlined once): the loop keeps a
// range [next, end) of queue positions in hand and refills it from the
// dispatch of the mode.  Bounded: each queue segment takes at most
// tile_cap + 1 pops, flat and per-task ranges advance every refill.
template <typename T, class Run>
__device__ __forceinline__ void for_each_task(const KArgs<T>& a, int mode, Run&& run) {
    const int wave = threadIdx.x / WAVE;
    const int64_t nt = (int64_t)*a.ntask;
    // an empty task list (a density fix-up pass with nothing flagged) ends
    // before any wavefront pops the shared counter
    if (nt <= 0) return;
    const bool queue = mode == MODE_QUEUE;
    const int qc = a.qchunk > 0 ? a.qchunk : QCHUNK;
    const bool split = queue && a.xcd_split;
    const int nseg = split ? NXCD : 1;
    const int x0 = split ? xcc_id() % NXCD : 0;
    int y = 0;         // queue: segments left behind
    int64_t pops = 0;  // queue: pops on the current segment
    bool pre = false;  // queue: a pop of the current segment is in flight
    int pv = 0;
    int64_t next = 0, end = 0;
    int64_t flat = blockIdx.x * (int64_t)WPB + wave;
    const int64_t fstep = (int64_t)gridDim.x * WPB;
    bool once = wave == 0;
    const int64_t guard_max = 2 * nt + (int64_t)nseg * (a.tile_cap + 2) + 2;
    for (int64_t guard = 0; guard < guard_max; ++guard) {
        if (next >= end) {
            if (queue) {
                if (y >= nseg) break;
                const int x = (x0 + y) % NXCD;
                const int64_t b = split ? nt * x / NXCD : 0;
                const int64_t e = split ? nt * (x + 1) / NXCD : nt;
                unsigned long long* head = &a.queue[split ? x : 0];
                int t0 = pv;
                if (!pre && lane_id() == 0) t0 = (int)atomicAdd(head, (unsigned long long)qc);
                pre = false;
                const int64_t s0 = b + uniform(t0);
                if (s0 >= e || ++pops > a.tile_cap + 1) {
                    ++y;
                    pops = 0;
                    continue;
                }
                next = s0;
                end = min(s0 + qc, e);
                // the next pop goes out now; its latency hides behind these tasks
                if (lane_id() == 0) pv = (int)atomicAdd(head, (unsigned long long)qc);
                pre = true;
            } else if (mode == MODE_FLAT) {
                if (flat >= nt) break;
                next = flat;
                end = flat + 1;
                flat += fstep;
            } else {
                if (!once || a.task < 0 || a.task >= nt) break;
                once = false;
                next = a.task;
                end = next + 1;
            }
        }
        // per-task: the launch names the tile itself; otherwise a queue position
        run(mode == MODE_PER_TASK ? (int)next : (int)a.order[next]);
        ++next;
    }
}

// Launch a loop kernel (k(args, mode)) in one of the three modes: the
// persistent queue (grid = resident workgroups, tasks popped from a device
// counter), flat (the same grid, tasks dealt round-robin: a static schedule)
// or one launch per task (reads the tile count back: synchronises).
template <int LK, typename T, int CAP>
int launch_with(void (*kern)(KArgs<T>, int), KArgs<T> a, int mode, int queue_slot,
                hipStream_t s) {
    constexpr size_t WMS = sizeof(WaveMem<T, CAP, LoopNV<LK>::NV>);
    const size_t shm = WMS * WPB;
    static bool attr_set = false;
    if (!attr_set) {
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm) != hipSuccess)
            return -1;
        attr_set = true;
    }
    if (a.tile_cap <= 0) return 0;
    a.queue = a.cnt->queue[queue_slot];
    if (mode == MODE_QUEUE || mode == MODE_FLAT) {
        if (mode == MODE_QUEUE) launch_fill_u32(a.queue, 2 * NXCD, 0u, s);
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, WPB * WAVE,
                                                         shm) != hipSuccess)
            per_cu = 1;
        if (per_cu < 1) per_cu = 1;
        int64_t blocks = (int64_t)per_cu * device_cu_count();
        const int64_t need = (a.tile_cap + WPB - 1) / WPB;
        if (blocks > need) blocks = need;
        hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(WPB * WAVE), shm, s, a, mode);
    } else {
        unsigned long long nt = 0;
        if (hipMemcpyAsync(&nt, a.ntask, sizeof nt, hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return -1;
        for (int64_t t = 0; t < (int64_t)nt; ++t) {
            a.task = (int32_t)t;
            hipLaunchKernelGGL(kern, dim3(1), dim3(WAVE), WMS, s, a, (int)MODE_PER_TASK);
        }
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

constexpr size_t LDS_LIMIT = 160 * 1024;

template <int LK, typename T, int CAP>
constexpr bool fits() {
    return WPB * sizeof(WaveMem<T, CAP, LoopNV<LK>::NV>) <= LDS_LIMIT;
}

}  // namespace swsph
