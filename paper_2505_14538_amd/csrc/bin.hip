// bin.hip -- device binning of particles into a hierarchy of cubic cells.
//
// The paper's solver splits each periodic box into cubic cells and works on
// self (one cell) and pair (two neighbouring cells) tasks, recursing in a
// cell tree down to cells of width ~H (Sec. 2.2, Sec. 2.2.2).  Here the cell
// hierarchy is implicit: particles are sorted by a Morton key of their cell
// on the finest grid (2^k cells per dimension in box b), so every coarser
// cubic cell is one contiguous range of the sorted array and its population
// is two lookups in the scanned fine histogram.
//
// Sort = counting sort on the key: histogram with atomics (which also hands
// each particle a slot inside its cell), exclusive scan, scatter, and a
// deterministic fix-up that orders the particles of each fine cell by their
// input index (so the result is independent of atomic timing).
#include <algorithm>

#include "launch.h"

namespace swsph {

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_copy_u64(unsigned long long* dst, const unsigned long long* src) {
    if (threadIdx.x == 0) *dst = *src;
}

void launch_copy_u64(unsigned long long* dst, const unsigned long long* src, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, s, dst, src);
}

void launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, n, v);
}

// ------------------------------------------------------------------ keys

template <typename T>
__global__ void k_keys(int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                       const T* __restrict__ z, const int32_t* __restrict__ box_id,
                       int32_t n_box, const BoxInfo* __restrict__ boxtab,
                       uint32_t* __restrict__ keys, int32_t* __restrict__ slot,
                       int32_t* __restrict__ fine_count, Counters* __restrict__ cnt) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    int b = box_id ? box_id[p] : 0;
    if (b < 0 || b >= n_box) {
        latch(cnt, SWSPH_ST_DOMAIN);
        b = b < 0 ? 0 : n_box - 1;
    }
    const BoxInfo bi = boxtab[b];
    const T L = (T)bi.L;
    T c[3] = {x[p], y[p], z[p]};
    const int q = 1 << bi.k;
    const T inv_w = (T)q / L;
    uint32_t ci[3];
    bool bad = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T v = c[d];
        if (!(v >= (T)0 && v < L)) bad = true;
        T f = v * inv_w;
        int k = (int)f;  // v >= 0: truncation is floor
        if (!(f >= (T)0)) k = 0;
        if (k >= q) k = q - 1;
        ci[d] = (uint32_t)k;
    }
    if (bad) latch(cnt, SWSPH_ST_DOMAIN);
    uint32_t key = (uint32_t)bi.fine_off + morton3(ci[0], ci[1], ci[2]);
    keys[p] = key;
    slot[p] = atomicAdd(&fine_count[key], 1);
}

template <typename T>
void launch_keys(const swsph_particles* p, const BoxInfo* boxtab, uint32_t* keys,
                 int32_t* slot, int32_t* fine_count, Counters* cnt, hipStream_t s) {
    int64_t n = p->n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_keys<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       (const T*)p->x, (const T*)p->y, (const T*)p->z, p->box_id, p->n_box,
                       boxtab, keys, slot, fine_count, cnt);
}
template void launch_keys<float>(const swsph_particles*, const BoxInfo*, uint32_t*, int32_t*,
                                 int32_t*, Counters*, hipStream_t);
template void launch_keys<double>(const swsph_particles*, const BoxInfo*, uint32_t*, int32_t*,
                                  int32_t*, Counters*, hipStream_t);

// ------------------------------------------------------------------ scan
// Exclusive scan of int32 counts, n up to 2^31: blocks of 1024 threads x 4
// items; block totals scanned by one block (looping over chunks).

constexpr int SCAN_T = 1024;
constexpr int SCAN_I = 4;
constexpr int SCAN_B = SCAN_T * SCAN_I;

__device__ __forceinline__ int block_exclusive_scan(int v, int* sh, int& total) {
    // wave-level inclusive scan with shuffles, then across the 16 waves
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int w = lane < (int)(blockDim.x >> 6) ? sh[lane] : 0;
        int y = w;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int t = __shfl_up(y, o, 64);
            if (lane >= o) y += t;
        }
        if (lane < (int)(blockDim.x >> 6)) sh[lane] = y - w;
        if (lane == (int)(blockDim.x >> 6) - 1) sh[32] = y;
    }
    __syncthreads();
    int excl = sh[wid] + x - v;
    total = sh[32];
    __syncthreads();
    return excl;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                        int32_t* __restrict__ part) {
    __shared__ int sh[40];
    int64_t base = (int64_t)blockIdx.x * SCAN_B + threadIdx.x * SCAN_I;
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) s += (base + k < n) ? in[base + k] : 0;
    int total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_partials(int32_t* __restrict__ part, int64_t nb) {
    __shared__ int sh[40];
    int carry = 0;
    for (int64_t c = 0; c < nb; c += SCAN_T) {
        int64_t i = c + threadIdx.x;
        int v = i < nb ? part[i] : 0;
        int total;
        int e = block_exclusive_scan(v, sh, total);
        if (i < nb) part[i] = e + carry;
        carry += total;
    }
}

__global__ void __launch_bounds__(SCAN_T) k_scan_final(const int32_t* __restrict__ in, int64_t n,
                                                       const int32_t* __restrict__ part,
                                                       int32_t* __restrict__ out) {
    __shared__ int sh[40];
    int64_t base = (int64_t)blockIdx.x * SCAN_B + threadIdx.x * SCAN_I;
    int v[SCAN_I];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int total;
    int e = block_exclusive_scan(s, sh, total) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_I; ++k) {
        if (base + k < n) out[base + k] = e;
        e += v[k];
    }
    // out[n] = grand total
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_T - 1) out[n] = e;
}

int64_t scan_partials_needed(int64_t n) { return (n + SCAN_B - 1) / SCAN_B + 1; }

void launch_exclusive_scan(const int32_t* in, int64_t n, int32_t* part, int32_t* out,
                           hipStream_t s) {
    int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n, part);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(SCAN_T), 0, s, part, nb);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(SCAN_T), 0, s, in, n, part, out);
}

// The particles each box received (from the scanned fine histogram) against
// the counts the caller declared on the host.  A mismatch means box_id and
// box_count disagree: the bin stays self-consistent (every kernel derives a
// particle's box from its cell key), but the result is not what the caller
// described, so it is reported as SWSPH_ST_DOMAIN.
__global__ void k_box_check(int32_t n_box, const BoxInfo* __restrict__ boxtab,
                            const int32_t* __restrict__ cstart, Counters* __restrict__ cnt) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n_box; b += gridDim.x * blockDim.x) {
        const BoxInfo bi = boxtab[b];
        const int64_t fb = bi.fine_off, fe = fb + (int64_t(1) << (3 * bi.k));
        if ((int64_t)(cstart[fe] - cstart[fb]) != bi.count) latch(cnt, SWSPH_ST_DOMAIN);
    }
}

void launch_box_check(int32_t n_box, const BoxInfo* boxtab, const int32_t* cstart, Counters* cnt,
                      hipStream_t s) {
    const unsigned g = (unsigned)std::min<int64_t>((n_box + 255) / 256, 1024);
    hipLaunchKernelGGL(k_box_check, dim3(g > 0 ? g : 1), dim3(256), 0, s, n_box, boxtab, cstart,
                       cnt);
}

// ------------------------------------------------------- scatter + fix-up

__global__ void k_scatter(int64_t n, const uint32_t* __restrict__ keys,
                          const int32_t* __restrict__ slot, const int32_t* __restrict__ cstart,
                          int32_t* __restrict__ tmpidx) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    tmpidx[cstart[keys[p]] + slot[p]] = (int32_t)p;
}

// Inside each fine cell, order particles by input index: the final position
// of particle p is the cell start plus the number of the cell's particles
// with a smaller index.
constexpr int32_t STABLE_MAX = 1 << 16;  // fine-cell population handled in order

__global__ void k_stable(int64_t n, const uint32_t* __restrict__ keys,
                         const int32_t* __restrict__ cstart, const int32_t* __restrict__ tmpidx,
                         int32_t* __restrict__ perm, int32_t* __restrict__ rank,
                         Counters* __restrict__ cnt) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t p = tmpidx[s];
    uint32_t key = keys[p];
    int32_t beg = cstart[key], end = cstart[key + 1];
    int32_t r = (int32_t)(s - beg);  // slot order if the cell is too crowded
    if (end - beg <= STABLE_MAX) {
        r = 0;
        for (int32_t t = beg; t < end; ++t) r += tmpidx[t] < p;
    } else if (s == beg) {
        latch(cnt, SWSPH_ST_LOOPCAP);
    }
    perm[beg + r] = p;
    rank[p] = beg + r;
}

void launch_scatter_stable(int64_t n, const uint32_t* keys, const int32_t* slot,
                           const int32_t* cstart, int32_t* tmpidx, int32_t* perm,
                           int32_t* rank, Counters* cnt, hipStream_t s) {
    if (n <= 0) return;
    unsigned g = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_scatter, dim3(g), dim3(256), 0, s, n, keys, slot, cstart, tmpidx);
    hipLaunchKernelGGL(k_stable, dim3(g), dim3(256), 0, s, n, keys, cstart, tmpidx, perm, rank, cnt);
}

// ---------------------------------------------------------------- gather

// Sorted copies: pos4 = (x, y, z, m), vel4 = (vx, vy, vz, u), hs = h guess.
// Without a guess, h0 is the geometric mean of two estimates eta / cbrt(n)
// of the local number density n: (1) n = N_l / w_l^3 of the first enclosing
// cell (walking up from the fine cell) that holds at least 16 particles,
// blended with the child cell's estimate where that cell holds more than
// 32; (2) n = N / (3 w)^3 of the first block of 3 x 3 x 3 cells centred on
// the particle's cell (periodic) that holds at least 16, walking up from two
// levels below the level (1) stopped at (a block that fine rarely holds 16
// when the particle's own cell one level up does not, and each level costs
// 27 cell-table reads).  A particle near a
// cell's face gets its density from its own cell only in (1) and from a
// neighbourhood about itself in (2); on the clustered 128^3 set (a host
// simulation against the solved h) the mean gives density tiles whose root
// lies beyond their staged radius 4x less often (3.1 % -> 0.8 %) for 1.4 %
// more staged volume.
__device__ inline double block_estimate(const BoxInfo& bi, uint32_t mort, int k, int top,
                                        const int32_t* __restrict__ cstart, double eta) {
    const uint32_t cx = compact3(mort), cy = compact3(mort >> 1), cz = compact3(mort >> 2);
    for (int lev = top; lev >= 0; --lev) {
        const int sh = k - lev;
        const uint32_t q = 1u << lev;
        const uint32_t bx = cx >> sh, by = cy >> sh, bz = cz >> sh;
        int64_t tot = 0;
        for (int d = 0; d < 27; ++d) {
            const uint32_t ox = (bx + q + (uint32_t)(d % 3) - 1u) & (q - 1u);
            const uint32_t oy = (by + q + (uint32_t)((d / 3) % 3) - 1u) & (q - 1u);
            const uint32_t oz = (bz + q + (uint32_t)(d / 9) - 1u) & (q - 1u);
            const int64_t fb = bi.fine_off + ((int64_t)morton3(ox, oy, oz) << (3 * sh));
            tot += cstart[fb + ((int64_t)1 << (3 * sh))] - cstart[fb];
        }
        if (tot >= 16 || lev == 0) {
            const double w = bi.L / (double)q;
            return eta * 3.0 * w / cbrt((double)(tot > 0 ? tot : 1));
        }
    }
    return 0.0;
}

template <typename T>
__global__ void k_gather(int64_t n, const T* __restrict__ x, const T* __restrict__ y,
                         const T* __restrict__ z, const T* __restrict__ vx,
                         const T* __restrict__ vy, const T* __restrict__ vz,
                         const T* __restrict__ u, const T* __restrict__ m,
                         const T* __restrict__ hin, int32_t n_box,
                         const BoxInfo* __restrict__ boxtab, const uint32_t* __restrict__ keys,
                         const int32_t* __restrict__ cstart, const int32_t* __restrict__ perm,
                         double eta, V4<T>* __restrict__ pos4, V4<T>* __restrict__ vel4,
                         T* __restrict__ hs) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t p = perm[s];
    V4<T> a, b;
    a.x = x[p]; a.y = y[p]; a.z = z[p]; a.w = m[p];
    b.x = vx[p]; b.y = vy[p]; b.z = vz[p]; b.w = u ? u[p] : (T)0;
    pos4[s] = a;
    vel4[s] = b;
    T h;
    if (hin) {
        h = hin[p];
    } else {
        const uint32_t key = keys[p];
        const BoxInfo bi = boxtab[box_of_key(key, n_box, boxtab)];
        uint32_t mort = key - (uint32_t)bi.fine_off;
        const int k = bi.k < 10 ? bi.k : 10;
        int lev = k;
        int64_t cntl = 0, child = 0;
        for (; lev >= 0; --lev) {
            int sh = 3 * (k - lev);
            int64_t beg = bi.fine_off + (int64_t)((mort >> sh) << sh);
            int64_t end = beg + (int64_t(1) << sh);
            child = cntl;
            cntl = cstart[end] - cstart[beg];
            if (cntl >= 16) break;
        }
        if (lev < 0) lev = 0;
        double w = bi.L / (double)(1 << lev);
        double hg = eta * w / cbrt((double)(cntl > 0 ? cntl : 1));
        if (cntl > 32 && lev < k) {
            // the enclosing cell is much fuller than the particle's own
            // (a clump elsewhere in it): meet the estimate of the child cell
            // half way (geometric mean), which halves the tiles whose root
            // lies beyond their staged neighbourhood
            const double hc = eta * 0.5 * w / cbrt((double)(child > 0 ? child : 1));
            hg = sqrt(hg * hc);
        }
        const double hb = block_estimate(bi, mort, k, lev + 2 < k ? lev + 2 : k, cstart, eta);
        if (hb > 0.0) hg = sqrt(hg * hb);
        h = (T)hg;
    }
    hs[s] = h;
}

template <typename T>
void launch_gather(const swsph_particles* p, const BoxInfo* boxtab, const uint32_t* keys,
                   const int32_t* cstart, const int32_t* perm, double eta, void* pos4,
                   void* vel4, void* hs, hipStream_t s) {
    int64_t n = p->n;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       (const T*)p->x, (const T*)p->y, (const T*)p->z, (const T*)p->vx,
                       (const T*)p->vy, (const T*)p->vz, (const T*)p->u, (const T*)p->m,
                       (const T*)p->h, p->n_box, boxtab, keys, cstart, perm, eta,
                       (V4<T>*)pos4, (V4<T>*)vel4, (T*)hs);
}
template void launch_gather<float>(const swsph_particles*, const BoxInfo*, const uint32_t*,
                                   const int32_t*, const int32_t*, double, void*, void*, void*,
                                   hipStream_t);
template void launch_gather<double>(const swsph_particles*, const BoxInfo*, const uint32_t*,
                                    const int32_t*, const int32_t*, double, void*, void*, void*,
                                    hipStream_t);

// ----------------------------------------------------------------- tiles
// A tile (one task of the loops) is the coarsest cell of the box's cell
// tree that holds at most `tile` particles; a finest cell holding more is
// cut into runs of `tile`.  Tiles are cubes, so their bounding boxes are
// compact and their task lists short even where the particle density
// changes by orders of magnitude; they come out in Morton order per box.
// Built in three passes: flag the first particle of every tile, scan the
// flags (tile index), write the tiles.  The tile count stays on the device;
// kernels over tiles loop up to it.  The density loop may use its own tile
// size.

// Sorted range [cbeg, cend) of the tile cell of binned particle s.
__device__ __forceinline__ void tile_cell(int64_t s, const BoxInfo& bi, uint32_t mort,
                                          const int32_t* __restrict__ cstart, int32_t tile,
                                          int64_t& cbeg, int64_t& cend) {
    const int k = bi.k;
    for (int l = 0; l <= k; ++l) {
        const int sh = 3 * (k - l);
        const int64_t fb = bi.fine_off + (int64_t)((mort >> sh) << sh);
        cbeg = cstart[fb];
        cend = cstart[fb + (int64_t(1) << sh)];
        if (cend - cbeg <= tile) return;
    }
}

__global__ void k_tile_flags(int64_t n, int32_t n_box, const BoxInfo* __restrict__ boxtab,
                             const uint32_t* __restrict__ keys, const int32_t* __restrict__ perm,
                             const int32_t* __restrict__ cstart, int32_t tile,
                             int32_t* __restrict__ flag) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint32_t key = keys[perm[s]];
    const BoxInfo bi = boxtab[box_of_key(key, n_box, boxtab)];
    const uint32_t mort = key - (uint32_t)bi.fine_off;
    int64_t cbeg = s, cend = s + 1;
    tile_cell(s, bi, mort, cstart, tile, cbeg, cend);
    flag[s] = ((s - cbeg) % tile) == 0 ? 1 : 0;
}

__global__ void k_tile_make(int64_t n, int32_t n_box, const BoxInfo* __restrict__ boxtab,
                            const uint32_t* __restrict__ keys, const int32_t* __restrict__ perm,
                            const int32_t* __restrict__ cstart, int32_t tile,
                            const int32_t* __restrict__ flag, const int32_t* __restrict__ tidx,
                            Tile* __restrict__ tiles, unsigned long long* __restrict__ ntiles) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    if (s == n - 1) *ntiles = (unsigned long long)tidx[n];
    if (!flag[s]) return;
    const uint32_t key = keys[perm[s]];
    const int b = box_of_key(key, n_box, boxtab);
    const BoxInfo bi = boxtab[b];
    const uint32_t mort = key - (uint32_t)bi.fine_off;
    int64_t cbeg = s, cend = s + 1;
    tile_cell(s, bi, mort, cstart, tile, cbeg, cend);
    Tile tl;
    tl.begin = (int32_t)s;
    tl.count = (int32_t)min((int64_t)tile, cend - s);
    tl.box = b;
    tl.flags = 0;
    tiles[tidx[s]] = tl;
}

// A coordinate narrowed to float without moving it inward: lo bounds round
// down, hi bounds up (exact for float data; for double data the float box
// still contains every particle, so distances to it never exceed the true
// ones and no cull built on it can drop a pair at the support edge).
__device__ __forceinline__ float narrow_lo(float v) { return v; }
__device__ __forceinline__ float narrow_hi(float v) { return v; }
__device__ __forceinline__ float narrow_lo(double v) {
    const float f = (float)v;
    return (double)f > v ? nextafterf(f, -INFINITY) : f;
}
__device__ __forceinline__ float narrow_hi(double v) {
    const float f = (float)v;
    return (double)f < v ? nextafterf(f, INFINITY) : f;
}

// The bounding box and largest h of each tile's particles.
template <typename T>
__global__ void k_tile_bounds(const V4<T>* __restrict__ pos4, const T* __restrict__ hs,
                              Tile* __restrict__ tiles, int32_t* __restrict__ order,
                              const unsigned long long* __restrict__ ntiles) {
    // one thread per tile (a tile holds at most 64 consecutive particles;
    // min and max are exact in any order)
    const int64_t nt = (int64_t)*ntiles;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += stride) {
        Tile tl = tiles[t];
        float lx = 3.0e38f, ly = 3.0e38f, lz = 3.0e38f;
        float ux = -3.0e38f, uy = -3.0e38f, uz = -3.0e38f, hm = 0.0f;
        const int cnt = tl.count < 64 ? tl.count : 64;
        for (int k = 0; k < cnt; ++k) {
            const V4<T> a = pos4[tl.begin + k];
            lx = fminf(lx, narrow_lo(a.x)); ly = fminf(ly, narrow_lo(a.y));
            lz = fminf(lz, narrow_lo(a.z));
            ux = fmaxf(ux, narrow_hi(a.x)); uy = fmaxf(uy, narrow_hi(a.y));
            uz = fmaxf(uz, narrow_hi(a.z));
            hm = fmaxf(hm, (float)hs[tl.begin + k]);
        }
        tl.lo[0] = lx; tl.lo[1] = ly; tl.lo[2] = lz;
        tl.hi[0] = ux; tl.hi[1] = uy; tl.hi[2] = uz;
        tl.hmax = hm;
        tl.cost = (float)tl.count;
        tiles[t] = tl;
        order[t] = (int32_t)t;
    }
}

// Blocks for a grid-stride launch of one wavefront per item.
unsigned wave_grid(int64_t items, int wpb) {
    int64_t b = (items + wpb - 1) / wpb;
    const int64_t cap = (int64_t)device_cu_count() * 16;
    if (b > cap) b = cap;
    return (unsigned)(b > 0 ? b : 1);
}

template <typename T>
static void make_tile_set(const BinPtrs& b, int32_t tile, Tile* tiles, int32_t* order,
                          unsigned long long* ntiles, hipStream_t s) {
    const unsigned g = (unsigned)((b.n + 255) / 256);
    hipLaunchKernelGGL(k_tile_flags, dim3(g), dim3(256), 0, s, b.n, b.n_box, b.boxtab, b.keys,
                       b.perm, b.cstart, tile, b.slot);
    launch_exclusive_scan(b.slot, b.n, b.scan_part, b.tmpidx, s);
    hipLaunchKernelGGL(k_tile_make, dim3(g), dim3(256), 0, s, b.n, b.n_box, b.boxtab, b.keys,
                       b.perm, b.cstart, tile, b.slot, b.tmpidx, tiles, ntiles);
    hipLaunchKernelGGL(k_tile_bounds<T>, dim3((unsigned)((b.tile_cap + 255) / 256)), dim3(256), 0, s,
                       (const V4<T>*)b.pos4, (const T*)b.hs, tiles, order,
                       (const unsigned long long*)ntiles);
}

// Parent of each density tile: the gradient/force tile containing its
// particles (cells nest, and both sets follow the same Morton order), read
// from the gradient/force tile scan at the tile's first particle.
__global__ void k_dparent(const Tile* __restrict__ tiles_d, const unsigned long long* __restrict__ ntd,
                          const int32_t* __restrict__ flag, const int32_t* __restrict__ tidx,
                          int32_t* __restrict__ dparent) {
    const int64_t nt = (int64_t)*ntd;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += nth) {
        const int32_t s = tiles_d[t].begin;
        dparent[t] = tidx[s] + flag[s] - 1;
    }
}

template <typename T>
void launch_make_tiles(const BinPtrs& b, hipStream_t s) {
    if (b.n <= 0) return;
    if (b.tiles_d != b.tiles) {
        make_tile_set<T>(b, b.tile_d, b.tiles_d, b.order_d, &b.cnt->n_tiles_d, s);
        make_tile_set<T>(b, b.tile, b.tiles, b.order, &b.cnt->n_tiles, s);
        // groups need density tiles inside gradient/force tiles: smaller ones
        if (b.tile_d < b.tile)
            hipLaunchKernelGGL(k_dparent, dim3(wave_grid(b.tile_cap, 4)), dim3(256), 0, s,
                               (const Tile*)b.tiles_d, (const unsigned long long*)&b.cnt->n_tiles_d,
                               (const int32_t*)b.slot, (const int32_t*)b.tmpidx, b.dparent);
    } else {
        make_tile_set<T>(b, b.tile, b.tiles, b.order, &b.cnt->n_tiles, s);
        launch_copy_u64(&b.cnt->n_tiles_d, &b.cnt->n_tiles, s);
    }
}
template void launch_make_tiles<float>(const BinPtrs&, hipStream_t);
template void launch_make_tiles<double>(const BinPtrs&, hipStream_t);

// ------------------------------------------------------ unsort of outputs

// out[p] = in[rank[p]] for the original particle p.
template <typename T>
__global__ void k_unsort(int64_t n, const int32_t* __restrict__ rank, const T* __restrict__ in,
                         T* __restrict__ out) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < n) out[p] = in[rank[p]];
}
template <typename T>
void launch_unsort(int64_t n, const int32_t* rank, const void* in, void* out, hipStream_t s) {
    if (n <= 0 || !out) return;
    hipLaunchKernelGGL(k_unsort<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, rank,
                       (const T*)in, (T*)out);
}
template void launch_unsort<float>(int64_t, const int32_t*, const void*, void*, hipStream_t);
template void launch_unsort<double>(int64_t, const int32_t*, const void*, void*, hipStream_t);
template void launch_unsort<int32_t>(int64_t, const int32_t*, const void*, void*, hipStream_t);

// Several arrays of one type in one launch (null outputs are skipped).
template <typename T>
__global__ void k_unsort_multi(int64_t n, const int32_t* __restrict__ rank, UnsortSet set) {
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t r = rank[p];
    for (int k = 0; k < set.k; ++k)
        if (set.out[k]) ((T*)set.out[k])[p] = ((const T*)set.in[k])[r];
}
template <typename T>
void launch_unsort_multi(int64_t n, const int32_t* rank, const UnsortSet& set, hipStream_t s) {
    if (n <= 0 || set.k <= 0) return;
    hipLaunchKernelGGL(k_unsort_multi<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       rank, set);
}
template void launch_unsort_multi<float>(int64_t, const int32_t*, const UnsortSet&, hipStream_t);
template void launch_unsort_multi<double>(int64_t, const int32_t*, const UnsortSet&, hipStream_t);
template void launch_unsort_multi<int32_t>(int64_t, const int32_t*, const UnsortSet&, hipStream_t);

// in-order -> sorted: out[s] = in[perm[s]]
template <typename T>
__global__ void k_sortcopy(int64_t n, const int32_t* __restrict__ perm, const T* __restrict__ in,
                           T* __restrict__ out) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s < n) out[s] = in[perm[s]];
}
template <typename T>
void launch_sortcopy(int64_t n, const int32_t* perm, const void* in, void* out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_sortcopy<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, perm,
                       (const T*)in, (T*)out);
}
template void launch_sortcopy<float>(int64_t, const int32_t*, const void*, void*, hipStream_t);
template void launch_sortcopy<double>(int64_t, const int32_t*, const void*, void*, hipStream_t);

}  // namespace swsph
