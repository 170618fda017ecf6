// adjoint.hip -- reverse mode of density -> force (hand-written adjoint).
//
// Loss L = sum_i gA_i . a_i + gU_i du_i/dt with the force loop of
// Sec. 2.1.4 (Eq. 17-18 + the viscosity of Eq. 7, 9-11) applied to the
// density loop of Sec. 2.1.2 (rho, drho/dh, f = 1/Omega from Eq. 8, and h
// defined by h^3 n(h) = eta^3).  Gradients with respect to positions,
// velocities, internal energies and masses.  Nothing per pair is stored:
// every pass recomputes the pair geometry.
//
//   pass A (pairs r < max(H_i, H_j)): for particle k, the terms of both
//     ordered pairs (k, j) and (j, k) of the force loop: dL/dx (through
//     r and the unit vector), dL/dv, dL/dm (k as the neighbour), and the
//     per-particle adjoints of A_k, f_k, c_k, rho_k (viscosity) and h_k
//     (through dW/dr at h_k);
//   pass B (per particle): A = f (gamma-1) u / rho, c = sqrt(gamma (gamma-1) u),
//     f = 1/Omega, Omega = 1 + h rho'/(3 rho): adjoints of u (final), rho,
//     rho' = drho/dh and h;
//   pass C (pairs): the density sums rho_k = sum_j m_j W(r, h_k) and
//     rho'_k = sum_j m_j dW/dh(r, h_k): dL/dx, dL/dm (k inside a neighbour's
//     sums, self term included) and the h_k term; then
//     lambda_k = hbar_k / (dG_k/dh) for G_k = h_k^3 n_k(h_k);
//   pass D (pairs): implicit function theorem on G_k = eta^3:
//     dL/dx_k -= sum over G_i depending on x_k of lambda_i dG_i/dx_k.
#include "loops_common.h"

namespace swsph {

// adjoint scratch (arrays of n, binned order)
enum {
    AJ_W4 = 0,       // V4: dL/da (3), dL/ddu  (occupies 4 arrays)
    AJ_RHODH = 4, AJ_WC = 5, AJ_WCDH = 6,
    AJ_GX = 7,       // 3 arrays
    AJ_GV = 10,      // 3 arrays
    AJ_GM = 13, AJ_GU = 14, AJ_GA = 15, AJ_GF = 16, AJ_GC = 17, AJ_GRHO = 18, AJ_GH = 19,
    AJ_GRHOP = 20, AJ_LAMBDA = 21,
    AJ_AUXC = 22,    // V4 (m, rho_bar, rho'_bar, 1/H)  (4 arrays)
    AJ_AUXD = 26,    // V4 (lambda h^3, 1/H, 0, 0)       (4 arrays)
    AJ_COUNT = 30
};

template <typename T> __device__ __forceinline__ T m4_w(T q) {
    const T t = (T)1 - q;
    return q < (T)0.5 ? (T)1 + q * q * ((T)6 * q - (T)6) : (T)2 * t * t * t;
}
template <typename T> __device__ __forceinline__ T m4_d2w(T q) {
    return q < (T)0.5 ? (T)36 * q - (T)12 : (T)12 * ((T)1 - q);
}

template <typename T> struct AdjPtrs {
    T* base;
    int64_t n;
    __device__ __forceinline__ T* arr(int k) const { return base + (int64_t)k * adj_stride(n); }
};

// ------------------------------------------------------------------ pass A

template <typename T, int CAP>
__device__ void adja_tile(WaveMem<T, CAP, 5>& m, const KArgs<T>& a, int t) {
    Tile tl = a.tiles[t];
    tl.begin = uniform(tl.begin);
    tl.count = uniform(tl.count);
    tl.box = uniform(tl.box);
    if (tl.count <= 0) return;
    const int lane = lane_id();
    const LaneMap q = lane_map(tl.count);
    const int js = q.js, S = q.S;
    const bool act = q.used();
    const bool lead = act && js == 0;  // writes the results of its i-particle
    const int i = tl.begin + (act ? q.li : 0);
    const BoxInfo bi = a.boxtab[tl.box];
    const V4<T> pi = a.pos4[i];
    const V4<T> vi = a.vel4[i];
    const V4<T> di = a.dens4[i];  // (rho, f, c, A)
    const V4<T> wi = a.aux4[i];   // (dL/dax, dL/day, dL/daz, dL/ddu)
    const T h = a.hs[i];
    const TileGeom g = geom_of(tl);
    const T eps = a.eps;
    const T H = mul_unfused(eps, h);
    const T H2 = act ? mul_unfused(H, H) : (T)-1;
    const T invH = (T)1 / H;
    const T cn = (T)(8.0 / PI_D);
    const T iH4 = invH * invH * invH * invH, iH5 = iH4 * invH;
    const T rhoi = di.x, fi = di.y, ci = di.z, Ai = di.w, mi = pi.w;
    const bool visc = (a.flags & SWSPH_NO_VISC) == 0;
    const T alpha = a.alpha, beta = a.beta;
    T gx = 0, gy = 0, gz = 0, gvx = 0, gvy = 0, gvz = 0;
    T gm = 0, gA = 0, gf = 0, gc = 0, grho = 0, gh = 0;
    // pairs with r = 0 (the self pair, coincident particles) contribute nothing
    auto test = [&](int k, bool ok) {
        const V4<T> s0 = m.s[0][k];
        const T r2 = dist2_unfused(pi.x - s0.x, pi.y - s0.y, pi.z - s0.z);
        return ok && act && r2 < max(H2, s0.w) && r2 > (T)0;
    };
    auto body = [&](int k) {
        const V4<T> s0 = m.s[0][k];
        const T dx = pi.x - s0.x, dy = pi.y - s0.y, dz = pi.z - s0.z;
        const T r2 = dist2_unfused(dx, dy, dz);
        const T H2j = s0.w;
        const V4<T> s1 = m.s[1][k];  // v_j, c_j
        const V4<T> s2 = m.s[2][k];  // m_j, A_j, f_j, 1/H_j
        const V4<T> s3 = m.s[3][k];  // rho_j, w_j
        const T ej = m.s[4][k].x;
        const T inv_r = fast_rsqrt(r2);
        const T r = r2 * inv_r;
        const T ex = dx * inv_r, ey = dy * inv_r, ez = dz * inv_r;
        // kernel at h_i: dW/dr, d2W/dr2, d2W/dh dr
        T gi = 0, gri = 0, ghi = 0;
        if (r2 < H2) {
            const T q = r * invH, dw = m4_dw(q), d2 = m4_d2w(q);
            gi = cn * iH4 * dw;
            gri = cn * iH5 * d2;
            ghi = -cn * eps * iH5 * ((T)4 * dw + q * d2);
        }
        T gj = 0, grj = 0;
        if (r2 < H2j) {
            const T ihj = s2.w;
            const T q = r * ihj, ih4 = ihj * ihj * ihj * ihj;
            gj = cn * ih4 * m4_dw(q);
            grj = cn * ih4 * ihj * m4_d2w(q);
        }
        const T mj = s2.x, Aj = s2.y, fj = s2.z, rhoj = s3.x;
        const T vxr = vi.x - s1.x, vyr = vi.y - s1.y, vzr = vi.z - s1.z;
        const T vdote = vxr * ex + vyr * ey + vzr * ez;
        const bool neg = vdote < (T)0;
        const T mu = neg ? vdote : (T)0;
        T nu = 0, dnu_dmu = 0, dnu_dc = 0, dnu_drho = 0;
        if (visc) {
            const T rs = rhoi + rhoj;
            const T vs = ci + s1.w - beta * mu;
            nu = -alpha * mu * vs / rs;
            dnu_dmu = -alpha * (vs - beta * mu) / rs;
            dnu_dc = -alpha * mu / rs;
            dnu_drho = -nu / rs;
        }
        const T Gs = fi * gi + fj * gj;
        const T Fn = Ai * gi + Aj * gj + (T)0.5 * nu * Gs;
        // ordered pair (i, j): weights of i, neighbour mass m_j
        const T p1 = wi.x * ex + wi.y * ey + wi.z * ez;
        const T Dn1 = Ai * gi + (T)0.25 * nu * Gs;
        const T k1 = (T)-0.5 * p1 + (T)0.25 * wi.w * vdote;
        gA += mj * gi * (wi.w * vdote - p1);
        gf += mj * nu * gi * k1;
        const T nub1 = mj * Gs * k1;
        const T gbi1 = mj * (-p1 * (Ai + (T)0.5 * nu * fi) + wi.w * vdote * (Ai + (T)0.25 * nu * fi));
        const T gbj1 = mj * (-p1 * (Aj + (T)0.5 * nu * fj) + wi.w * vdote * (T)0.25 * nu * fj);
        const T vdb1 = wi.w * mj * Dn1 + (neg ? nub1 * dnu_dmu : (T)0);
        // ordered pair (j, i): weights of j, neighbour mass m_i, unit vector -e
        const T p2 = -(s3.y * ex + s3.z * ey + s3.w * ez);
        const T Dn2 = Aj * gj + (T)0.25 * nu * Gs;
        const T k2 = (T)-0.5 * p2 + (T)0.25 * ej * vdote;
        gA += -p2 * mi * gi;
        gf += mi * nu * gi * k2;
        const T nub2 = mi * Gs * k2;
        const T gbi2 = mi * (-p2 * (Ai + (T)0.5 * nu * fi) + ej * vdote * (T)0.25 * nu * fi);
        const T gbj2 = mi * (-p2 * (Aj + (T)0.5 * nu * fj) + ej * vdote * (Aj + (T)0.25 * nu * fj));
        const T vdb2 = ej * mi * Dn2 + (neg ? nub2 * dnu_dmu : (T)0);
        gm += -p2 * Fn + ej * Dn2 * vdote;
        gc += (nub1 + nub2) * dnu_dc;
        grho += (nub1 + nub2) * dnu_drho;
        gh += (gbi1 + gbi2) * ghi;
        // geometry: r (through the kernel derivatives) and the unit vector
        const T rb = (gbi1 + gbi2) * gri + (gbj1 + gbj2) * grj;
        const T vdb = vdb1 + vdb2;
        const T Ex = -mj * Fn * wi.x + mi * Fn * s3.y + vdb * vxr;
        const T Ey = -mj * Fn * wi.y + mi * Fn * s3.z + vdb * vyr;
        const T Ez = -mj * Fn * wi.z + mi * Fn * s3.w + vdb * vzr;
        const T Ee = Ex * ex + Ey * ey + Ez * ez;
        gx += rb * ex + (Ex - Ee * ex) * inv_r;
        gy += rb * ey + (Ey - Ee * ey) * inv_r;
        gz += rb * ez + (Ez - Ee * ez) * inv_r;
        gvx += vdb * ex;
        gvy += vdb * ey;
        gvz += vdb * ez;
    };
    auto sweep = [&](int ns) { pair_loop(m, ns, js, S, test, body); };
    int flushes = 0;
    const T R = (T)a.trad[t];
    const int ns = stage_tile<L_ADJA, T, CAP>(m, a, t, bi, g, R * R, flushes, sweep);
    sweep(ns);
    gx = stream_sum(gx, q); gy = stream_sum(gy, q); gz = stream_sum(gz, q);
    gvx = stream_sum(gvx, q); gvy = stream_sum(gvy, q); gvz = stream_sum(gvz, q);
    gm = stream_sum(gm, q); gA = stream_sum(gA, q); gf = stream_sum(gf, q);
    gc = stream_sum(gc, q); grho = stream_sum(grho, q); gh = stream_sum(gh, q);
    if (lead) {
        AdjPtrs<T> J{a.out, a.n};
        J.arr(AJ_GX)[i] = gx;
        J.arr(AJ_GX + 1)[i] = gy;
        J.arr(AJ_GX + 2)[i] = gz;
        J.arr(AJ_GV)[i] = gvx;
        J.arr(AJ_GV + 1)[i] = gvy;
        J.arr(AJ_GV + 2)[i] = gvz;
        J.arr(AJ_GM)[i] = gm;
        J.arr(AJ_GA)[i] = gA;
        J.arr(AJ_GF)[i] = gf;
        J.arr(AJ_GC)[i] = gc;
        J.arr(AJ_GRHO)[i] = grho;
        J.arr(AJ_GH)[i] = gh;
    }
}

// ------------------------------------------------------------------ pass C

template <typename T, int CAP>
__device__ void adjc_tile(WaveMem<T, CAP, 2>& m, const KArgs<T>& a, int t) {
    Tile tl = a.tiles[t];
    tl.begin = uniform(tl.begin);
    tl.count = uniform(tl.count);
    tl.box = uniform(tl.box);
    if (tl.count <= 0) return;
    const int lane = lane_id();
    const LaneMap q = lane_map(tl.count);
    const int js = q.js, S = q.S;
    const bool act = q.used();
    const bool lead = act && js == 0;  // writes the results of its i-particle
    const int i = tl.begin + (act ? q.li : 0);
    const BoxInfo bi = a.boxtab[tl.box];
    const V4<T> pi = a.pos4[i];
    const T h = a.hs[i];
    const TileGeom g = geom_of(tl);
    const T eps = a.eps;
    const T H = mul_unfused(eps, h);
    const T H2 = act ? mul_unfused(H, H) : (T)-1;
    const T invH = (T)1 / H;
    const T cn = (T)(8.0 / PI_D);
    const T iH4 = invH * invH * invH * invH, iH5 = iH4 * invH;
    AdjPtrs<T> J{a.out, a.n};
    const V4<T> ai = a.aux4[i];  // (m_i, rho_bar_i, rho'_bar_i, 1/H_i)
    const T rb = ai.y, rpb = ai.z, mi = pi.w;
    T gx = 0, gy = 0, gz = 0, gm = 0, gh = 0;
    auto test = [&](int k, bool ok) {
        const V4<T> s0 = m.s[0][k];
        const T r2 = dist2_unfused(pi.x - s0.x, pi.y - s0.y, pi.z - s0.z);
        return ok && (r2 < H2 || (act && r2 < s0.w));
    };
    auto body = [&](int k) {
        const V4<T> s0 = m.s[0][k];
        const T dx = pi.x - s0.x, dy = pi.y - s0.y, dz = pi.z - s0.z;
        const T r2 = dist2_unfused(dx, dy, dz);
        const bool own = r2 < H2, rev = act && r2 < s0.w;
        const V4<T> s1 = m.s[1][k];  // (m_j, rho_bar_j, rho'_bar_j, 1/H_j)
        const T inv_r = r2 > (T)0 ? fast_rsqrt(r2) : (T)0;
        const T r = r2 * inv_r;
        T sx = 0;
        if (own) {
            const T q = r * invH, w = m4_w(q), dw = m4_dw(q), d2 = m4_d2w(q);
            const T Wh = -cn * eps * iH4 * ((T)3 * w + q * dw);
            const T Whh = cn * eps * eps * iH5 * ((T)12 * w + (T)8 * q * dw + q * q * d2);
            const T Wr = cn * iH4 * dw;
            const T Wrh = -cn * eps * iH5 * ((T)4 * dw + q * d2);
            gh += s1.x * (rb * Wh + rpb * Whh);
            sx += s1.x * (rb * Wr + rpb * Wrh);
        }
        if (rev) {
            const T ihj = s1.w;
            const T q = r * ihj, w = m4_w(q), dw = m4_dw(q), d2 = m4_d2w(q);
            const T ih3 = ihj * ihj * ihj, ih4 = ih3 * ihj, ih5 = ih4 * ihj;
            const T Wj = cn * ih3 * w;
            const T Whj = -cn * eps * ih4 * ((T)3 * w + q * dw);
            const T Wrj = cn * ih4 * dw;
            const T Wrhj = -cn * eps * ih5 * ((T)4 * dw + q * d2);
            gm += s1.y * Wj + s1.z * Whj;
            sx += mi * (s1.y * Wrj + s1.z * Wrhj);
        }
        gx += sx * dx * inv_r;
        gy += sx * dy * inv_r;
        gz += sx * dz * inv_r;
    };
    auto sweep = [&](int ns) { pair_loop(m, ns, js, S, test, body); };
    int flushes = 0;
    const T R = (T)a.trad[t];
    const int ns = stage_tile<L_ADJC, T, CAP>(m, a, t, bi, g, R * R, flushes, sweep);
    sweep(ns);
    gx = stream_sum(gx, q); gy = stream_sum(gy, q); gz = stream_sum(gz, q);
    gm = stream_sum(gm, q); gh = stream_sum(gh, q);
    if (lead) {
        J.arr(AJ_GX)[i] += gx;
        J.arr(AJ_GX + 1)[i] += gy;
        J.arr(AJ_GX + 2)[i] += gz;
        J.arr(AJ_GM)[i] += gm;
        const T hbar = J.arr(AJ_GH)[i] + gh;
        const T n = J.arr(AJ_WC)[i], ndh = J.arr(AJ_WCDH)[i];
        const T dG = (T)3 * h * h * n + h * h * h * ndh;
        const T lam = hbar / dG;
        J.arr(AJ_LAMBDA)[i] = lam;
        ((V4<T>*)J.arr(AJ_AUXD))[i] = V4<T>{lam * h * h * h, invH, (T)0, (T)0};
    }
}

// ------------------------------------------------------------------ pass D

template <typename T, int CAP>
__device__ void adjd_tile(WaveMem<T, CAP, 2>& m, const KArgs<T>& a, int t) {
    Tile tl = a.tiles[t];
    tl.begin = uniform(tl.begin);
    tl.count = uniform(tl.count);
    tl.box = uniform(tl.box);
    if (tl.count <= 0) return;
    const int lane = lane_id();
    const LaneMap q = lane_map(tl.count);
    const int js = q.js, S = q.S;
    const bool act = q.used();
    const bool lead = act && js == 0;  // writes the results of its i-particle
    const int i = tl.begin + (act ? q.li : 0);
    const BoxInfo bi = a.boxtab[tl.box];
    const V4<T> pi = a.pos4[i];
    const T h = a.hs[i];
    const TileGeom g = geom_of(tl);
    const T eps = a.eps;
    const T H = mul_unfused(eps, h);
    const T H2 = act ? mul_unfused(H, H) : (T)-1;
    const T invH = (T)1 / H;
    const T cn = (T)(8.0 / PI_D);
    const T iH4 = invH * invH * invH * invH;
    AdjPtrs<T> J{a.out, a.n};
    const T lhi = a.aux4[i].x;  // lambda_i h_i^3
    T gx = 0, gy = 0, gz = 0;
    auto test = [&](int k, bool ok) {
        const V4<T> s0 = m.s[0][k];
        const T r2 = dist2_unfused(pi.x - s0.x, pi.y - s0.y, pi.z - s0.z);
        return ok && (r2 < H2 || (act && r2 < s0.w)) && r2 > (T)0;
    };
    auto body = [&](int k) {
        const V4<T> s0 = m.s[0][k];
        const T dx = pi.x - s0.x, dy = pi.y - s0.y, dz = pi.z - s0.z;
        const T r2 = dist2_unfused(dx, dy, dz);
        const bool own = r2 < H2, rev = act && r2 < s0.w;
        const V4<T> s1 = m.s[1][k];  // (lambda_j h_j^3, 1/H_j)
        const T inv_r = fast_rsqrt(r2);
        const T r = r2 * inv_r;
        T c = 0;
        if (own) c += lhi * cn * iH4 * m4_dw(r * invH);
        if (rev) {
            const T ihj = s1.y;
            c += s1.x * cn * ihj * ihj * ihj * ihj * m4_dw(r * ihj);
        }
        gx -= c * dx * inv_r;
        gy -= c * dy * inv_r;
        gz -= c * dz * inv_r;
    };
    auto sweep = [&](int ns) { pair_loop(m, ns, js, S, test, body); };
    int flushes = 0;
    const T R = (T)a.trad[t];
    const int ns = stage_tile<L_ADJD, T, CAP>(m, a, t, bi, g, R * R, flushes, sweep);
    sweep(ns);
    gx = stream_sum(gx, q); gy = stream_sum(gy, q); gz = stream_sum(gz, q);
    if (lead) {
        J.arr(AJ_GX)[i] += gx;
        J.arr(AJ_GX + 1)[i] += gy;
        J.arr(AJ_GX + 2)[i] += gz;
    }
}

// ----------------------------------------------------------------- drivers

template <int LK, typename T, int CAP>
__global__ void __launch_bounds__(WPB * WAVE) k_adj(KArgs<T> a, int mode) {
    SWSPH_DYN_SHARED char smem[];
    constexpr size_t WMS = sizeof(WaveMem<T, CAP, LoopNV<LK>::NV>);
    const int wave = threadIdx.x / WAVE;
    char* wm = smem + wave * WMS;
    auto body = [&](int t) {
        if (LK == L_ADJA) adja_tile<T, CAP>(*(WaveMem<T, CAP, 5>*)wm, a, t);
        else if (LK == L_ADJC) adjc_tile<T, CAP>(*(WaveMem<T, CAP, 2>*)wm, a, t);
        else adjd_tile<T, CAP>(*(WaveMem<T, CAP, 2>*)wm, a, t);
    };
    for_each_task(a, mode, body);
}

template <int LK, typename T>
static int launch_adj(KArgs<T> a, int mode, int lds_cap, hipStream_t s) {
    if (lds_cap >= 256 && fits<LK, T, 256>())
        return launch_with<LK, T, 256>(k_adj<LK, T, 256>, a, mode, 3, s);
    static_assert(fits<LK, T, 128>(), "staging buffer does not fit");
    return launch_with<LK, T, 128>(k_adj<LK, T, 128>, a, mode, 3, s);
}

// Gather the loss gradients and the density results the adjoint needs.
template <typename T>
__global__ void k_adj_prep(int64_t n, const int32_t* __restrict__ perm, const T* __restrict__ gax,
                           const T* __restrict__ gay, const T* __restrict__ gaz,
                           const T* __restrict__ gdu, const T* __restrict__ rho_dh,
                           const T* __restrict__ wc, const T* __restrict__ wcdh, T* __restrict__ J) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t st = adj_stride(n);
    const int32_t p = perm[s];
    ((V4<T>*)J)[s] = V4<T>{gax[p], gay[p], gaz[p], gdu[p]};
    J[AJ_RHODH * st + s] = rho_dh[p];
    J[AJ_WC * st + s] = wc[p];
    J[AJ_WCDH * st + s] = wcdh[p];
}

// Pass B: chain through A, c, f = 1/Omega and Omega (per particle).
template <typename T>
__global__ void k_adj_b(int64_t n, const V4<T>* __restrict__ pos4, const V4<T>* __restrict__ vel4,
                        const V4<T>* __restrict__ dens4, const T* __restrict__ hs, T gamma, T eps,
                        T* __restrict__ J) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t st = adj_stride(n);
    const V4<T> d = dens4[s];  // (rho, f, c, A)
    const T u = vel4[s].w, h = hs[s], rho = d.x, f = d.y, c = d.z, A = d.w;
    const T rhop = J[AJ_RHODH * st + s];
    const T gA = J[AJ_GA * st + s];
    const T gm1 = gamma - (T)1;
    T gu = gA * f * gm1 / rho;
    if (c > (T)0) gu += J[AJ_GC * st + s] * gamma * gm1 / ((T)2 * c);
    const T gf = J[AJ_GF * st + s] + gA * gm1 * u / rho;
    T grho = J[AJ_GRHO * st + s] - gA * A / rho;
    const T gOm = -gf * f * f;
    const T gh = J[AJ_GH * st + s] + gOm * rhop / ((T)3 * rho);
    const T grhop = gOm * h / ((T)3 * rho);
    grho += -gOm * h * rhop / ((T)3 * rho * rho);
    J[AJ_GU * st + s] = gu;
    J[AJ_GRHO * st + s] = grho;
    J[AJ_GRHOP * st + s] = grhop;
    J[AJ_GH * st + s] = gh;
    ((V4<T>*)(J + AJ_AUXC * st))[s] = V4<T>{pos4[s].w, grho, grhop, (T)1 / (eps * h)};
}

template <typename T>
int launch_backward(const BinPtrs& b, const Scheme& sc, const swsph_force_grad* g,
                    const swsph_density_out* d, int lds_cap, hipStream_t s) {
    const int64_t n = b.n;
    if (n <= 0) return 0;
    T* J = (T*)b.adj;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    launch_prep_dens<T>(b, sc, d, s);
    hipLaunchKernelGGL(k_adj_prep<T>, dim3(blocks), dim3(256), 0, s, n, b.perm, (const T*)g->gax,
                       (const T*)g->gay, (const T*)g->gaz, (const T*)g->gdudt,
                       (const T*)d->rho_dh, (const T*)d->wcount, (const T*)d->wcount_dh, J);
    launch_hmax_pyramid<T>(b, sc, s);
    launch_tasks<T>(b, sc, 2, false, s);
    KArgs<T> a = make_args<T>(b, sc);
    a.out = J;
    const int mode = (sc.flags & SWSPH_FLAT_LAUNCH) ? MODE_FLAT : MODE_QUEUE;
    a.aux4 = (const V4<T>*)J;  // AJ_W4
    timer_begin(sc.timer, 3, s);
    int r = launch_adj<L_ADJA, T>(a, mode, lds_cap, s);
    timer_end(sc.timer, 3, s);
    hipLaunchKernelGGL(k_adj_b<T>, dim3(blocks), dim3(256), 0, s, n, (const V4<T>*)b.pos4,
                       (const V4<T>*)b.vel4, (const V4<T>*)b.dens4, (const T*)b.hs, (T)sc.gamma,
                       (T)sc.eps, J);
    a.aux4 = (const V4<T>*)(J + AJ_AUXC * adj_stride(n));
    r |= launch_adj<L_ADJC, T>(a, mode, lds_cap, s);
    a.aux4 = (const V4<T>*)(J + AJ_AUXD * adj_stride(n));
    r |= launch_adj<L_ADJD, T>(a, mode, lds_cap, s);
    return r;
}
template int launch_backward<float>(const BinPtrs&, const Scheme&, const swsph_force_grad*,
                                    const swsph_density_out*, int, hipStream_t);
template int launch_backward<double>(const BinPtrs&, const Scheme&, const swsph_force_grad*,
                                     const swsph_density_out*, int, hipStream_t);

int adj_arrays() { return AJ_COUNT; }

}  // namespace swsph
