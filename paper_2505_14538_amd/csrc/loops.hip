// loops.hip -- gfx950 kernels of the density loop and of the joint gradient
// and force loop.
//
// Work decomposition (MI355X-first; the paper's CUDA kernels are not shown
// and were written for V100/H100/L40, so nothing is carried over):
//   * task = one i-tile: a cell of the cell tree holding at most `tile`
//     binned particles (lanes map to i-slots x streams of a 64-wide
//     wavefront);
//   * the tile's task list (the particles of its own and neighbouring cells,
//     i.e. the paper's self and pair tasks, Sec. 2.2.2) comes from tasks.hip
//     as candidate entries (particle index and periodic-image code), already
//     culled against the tile box;
//   * the candidates are streamed through the lanes (coalesced entry reads,
//     one gather round trip per batch), culled by the loop's own radius and
//     staged in LDS (arrays of 4-vectors);
//   * every lane then runs over the staged j-particles (LDS broadcast reads)
//     and accumulates its own sums -- a gather, so no atomics and a fixed
//     summation order (results are bitwise reproducible);
//   * the density loop iterates Newton on h over the staged set; a lane whose
//     h outgrows the staged radius leaves its tile flagged for a fix-up pass
//     with a wider task list.
// Launch modes: a persistent kernel whose wavefronts pull tasks from a device
// queue, a flat launch (one wavefront per task) and one launch per task (the
// per-task offload baseline).  Every loop has a fixed upper bound.
#include <algorithm>

#include "loops_common.h"

namespace swsph {

// ------------------------------------------------------------ density tile
//
// The tile's candidates within the staged radius R of its box are staged in
// LDS (image position and binned index).  Every i-particle then gets its own
// list of the staged candidates within R of it -- one pass of distance
// tests; h is held below R / eps, so the lists hold every pair any sweep can
// reach -- and the Newton (Halley) sweeps evaluate the kernel over those
// lists with only the sums the step needs (n and its first two log-h
// derivatives).  One full sweep at the final h adds rho, its h-derivative,
// div v, curl v and the neighbour count, reading the partner's mass and
// velocity from global memory.  A tile whose candidates overflow the staging
// buffer (or whose lists overflow) tests the staged set again every sweep,
// staging it again as needed.
// Lanes: c i-slots of S contiguous streams (S a power of two), so the sums
// over a slot's streams are DPP butterflies.

// Step arithmetic of the Halley update: fast hardware reciprocal and
// exponential in FP32 (the iteration's stop test is exact, so their
// rounding only shapes the path to the root), the library functions in FP64.
__device__ __forceinline__ float step_rcp(float x) { return fast_rcp(x); }
__device__ __forceinline__ double step_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float step_exp(float x) { return __expf(x); }
__device__ __forceinline__ double step_exp(double x) { return exp(x); }

// SINGLE (the single-launch step): also write (rho, f, c, A) of each
// particle, and return 1 when some h needs a wider staged set, 2 when an
// iteration failed or some h has a support the box's early gradient/force
// lists may not cover (0 otherwise).
template <typename T, int CAP, bool SINGLE = false>
__device__ __forceinline__ int density_tile(WaveMem<T, CAP, 1>& m, const KArgs<T>& a, int t,
                                            WaveStats& ws, float Rset = 0.f) {
    Tile tl = a.tiles[t];
    tl.begin = uniform(tl.begin);
    tl.count = uniform(tl.count);
    tl.box = uniform(tl.box);
    if (tl.count <= 0) return 0;
    if (a.fixup && a.tflag[t] == 0) return 0;
    const int lane = lane_id();
    // A fix-up pass iterates only the particles an earlier pass left pending
    // (it stores their next guess negated); the others keep their results,
    // and the pending ones get all of the wavefront's streams.  A flagged
    // tile with none marked runs whole.
    int nsel = tl.count;
    unsigned long long selm = 0ull;
    if (a.fixup) {
        selm = ballot(lane < tl.count && a.hs[tl.begin + lane] < (T)0);
        if (selm) nsel = __popcll(selm);
    }
    const GroupMap q = group_map(nsel);
    const int js = q.js, S = q.S, c = q.c;
    const bool act = q.act;
    const bool lead = act && js == 0;  // writes the results of its i-particle
    int pos = q.li;  // the i-slot's particle within the tile
    if (selm) {
        unsigned long long mm = selm;
        for (int r = 0; r < q.li; ++r) mm &= mm - 1ull;
        pos = mm ? (int)__builtin_ctzll(mm) : 0;
    }
    const int i = tl.begin + pos;
    const BoxInfo bi = a.boxtab[tl.box];
    const V4<T> pi = a.pos4[i];
    T h = a.hs[i];
    if (h < (T)0) h = -h;
    const bool fixed = (a.flags & SWSPH_FIXED_H) != 0;
    // a fix-up pass over the pending particles stages around their box only
    // (recorded by the fix-up task build, whose list serves that box)
    TileGeom g = geom_of(tl);
    if (selm && a.fbox) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            g.lo[d] = a.fbox[6 * t + d];
            g.hi[d] = a.fbox[6 * t + 3 + d];
        }
    }
    const T Rcap = (T)(0.5f * (float)bi.L * (1.0f - 1e-6f));
    const T eps = a.eps;
    const T cnorm = (T)(8.0 / PI_D);
    // root of sum_j w(q_ij) = Tt  <=>  h^3 n(h) = eta^3
    const T Tt = a.eta * a.eta * a.eta * eps * eps * eps / cnorm;
    const T inv_Tt = (T)1 / Tt;
    const T tiny = (sizeof(T) == 4) ? (T)2.4e-7 : (T)4.5e-16;
    // staged radius: in a first pass over lists shared with the parent
    // gradient/force tile, the margin over this tile's largest guessed
    // support (formed as a list build forms it); else the tile's own radius
    T R;
    const bool shared = a.parent != nullptr && !a.fixup;
    if (shared) {
        const T hm = wave_max(act ? h : (T)0);
        const float Rcf = 0.5f * (float)bi.L * (1.0f - 1e-6f);
        float Rf = (float)(eps * hm * a.dmargin * (T)(1 + 4e-7));
        if (!(Rf < Rcf)) {
            if (a.dmargin == (T)1 && lane == 0) latch(a.cnt, SWSPH_ST_REACH);
            Rf = Rcf;
        }
        if (!(Rf > 0.f)) Rf = Rcf;
        if (SINGLE && Rset > Rf) Rf = Rset;  // a second run with a wider radius
        R = (T)Rf;
    } else {
        R = (T)a.trad[t];
    }
    const int lt = shared ? uniform(a.parent[t]) : t;  // whose list is staged
    const T hstage = R / eps;
    const T hedge = hstage * ((T)1 - (T)8 * tiny);  // largest h whose support is staged

    // a guess beyond the staged radius starts at its edge (the radius is
    // capped below half the box)
    if (!fixed && h > hedge) h = hedge;
    T lo_h = 0, hi_h = hstage;
    bool has_upper = false;
    bool conv = fixed || !act;
    bool pend = false, failed = false;
    T want = 0;
    int iters = a.fixup ? max(0, a.iout[a.n + i] < 0 ? -a.iout[a.n + i] : a.iout[a.n + i]) : 0;
    const int iters0 = iters;
    T S0 = 0, S1 = 0, S2 = 0, Sr = 0, Sdr = 0, Dv = 0, Cx = 0, Cy = 0, Cz = 0;
    int cnt = 0;
    unsigned long long tested = 0;      // per i-particle
    unsigned long long tested_lane = 0;  // list evaluations of this lane's slot (lead lanes)
    T H = eps * h;
    T H2 = act ? mul_unfused(H, H) : (T)-1;
    T invH = (T)1 / H;
    // Halley steps below ds_pred (in log h) are taken without a confirming
    // sweep when allowed: their error, about the step's cube, stays well
    // inside h_tol, and the full sweep at the new h checks the stop
    // criterion anyway (a particle that fails it iterates on)
    bool pred = false, allow_pred = false;
    const T ds_pred = cbrt((T)2 * a.h_tol);
    // a pair inside the support: sj the staged image position, pj and vj the
    // partner's pos4 (mass in w) and vel4; vi the particle's own velocity
    V4<T> vi{};
    auto body = [&](const V4<T>& sj, const V4<T>& pj, const V4<T>& vj) {
        const T dx = pi.x - sj.x, dy = pi.y - sj.y, dz = pi.z - sj.z;
        const T r2 = dist2_unfused(dx, dy, dz);
        const T inv_r = r2 > (T)0 ? fast_rsqrt(r2) : (T)0;
        const T qq = r2 * inv_r * invH;
        T w, s1, gq;
        m4_terms(qq, H * inv_r, w, s1, gq);
        S0 += w;
        S1 += s1;
        S2 += m4_q2w2(qq);
        Sr += pj.w * w;
        Sdr += pj.w * s1;
        const T ux = vi.x - vj.x, uy = vi.y - vj.y, uz = vi.z - vj.z;
        const T mg = pj.w * gq;
        Dv += mg * (ux * dx + uy * dy + uz * dz);
        Cx += mg * (uy * dz - uz * dy);
        Cy += mg * (uz * dx - ux * dz);
        Cz += mg * (ux * dy - uy * dx);
        ++cnt;
    };
    auto body_k = [&](int k) {
        const V4<T> sj = m.s[0][k];
        int j = as_int<T>(sj.w);
        if (j < 0 || j >= a.n) j = 0;  // cannot happen with a valid list
        body(sj, a.pos4[j], a.vel4[j]);
    };
    auto test = [&](int k, bool ok) {
        const V4<T> sj = m.s[0][k];
        return ok & (dist2_unfused(pi.x - sj.x, pi.y - sj.y, pi.z - sj.z) < H2);
    };
    auto sweep = [&](int ns) {
        pair_loop(m, ns, js, S, test, body_k);
        tested += (unsigned long long)ns;
    };
    auto zero = [&]() {
        S0 = S1 = S2 = Sr = Sdr = Dv = Cx = Cy = Cz = 0;
        cnt = 0;
    };
    // One Halley update per lane from the sums of the sweep at h (over the
    // streams of its i-particle).
    auto newton = [&](T S0r, T S1r, T S2r) {
        pred = false;
        if (conv || pend) return;
        const T G = S0r;
        if (fabs(G - Tt) <= a.h_tol * Tt) {
            conv = true;
            return;
        }
        // Halley step on F = log(G / target) over log h: G grows about as
        // h^3, so F is nearly linear in log h, and the third-order step (F'
        // from h dG/dh = 3 S0 - S1, F'' from the sum of q^2 w''(q) as well)
        // saves about half a sweep per particle over a Newton step on the
        // same function
        const T dl = (T)3 * S0r - S1r;
        if (G < Tt) lo_h = h; else { hi_h = h; has_upper = true; }
        const T iG = step_rcp(G);
        const T F = log1p((G - Tt) * inv_Tt);
        const T F1 = dl * iG;
        const T F2 = (S2r - dl) * iG - F1 * F1;
        const T den = (T)2 * F1 * F1 - F * F2;
        const T ds = den > (T)0 ? (T)-2 * F * F1 * step_rcp(den) : -F * step_rcp(F1);
        T hn = h * step_exp(ds);
        const bool ok = dl > (T)0 && hn > lo_h && hn < hi_h;
        if (!ok) hn = has_upper ? (T)0.5 * (lo_h + hi_h) : (T)2 * h;
        if (!has_upper && hn >= hedge) {
            // the step leaves the staged set: first try its edge; if the
            // root lies beyond, the tile gets a fix-up pass
            if (h < hedge) {
                h = hedge;
            } else if (R >= Rcap) {
                failed = true;
                conv = true;
            } else {
                // next radius from the local h^3 scaling of G (a Newton step
                // from below can overshoot far), grown at most 2x per pass
                pend = true;
                const T grow = (T)1.02 * cbrt(Tt / G);
                want = h * min((T)2, max((T)1.02, grow));
            }
        } else if (fabs(hn - h) <= tiny * h) {
            conv = true;
        } else {
            // a small accepted step leaves an error of order its cube
            // (Halley): the next sweep would only confirm it
            pred = allow_pred && ok && fabs(ds) <= ds_pred;
            h = hn;
        }
    };
    auto next_h = [&]() {
        H = eps * h;
        H2 = act ? mul_unfused(H, H) : (T)-1;
        invH = (T)1 / H;
    };
    const T R2 = R * R;
    int flushes = 0;
    int ns = stage_tile<L_DENS, T, CAP>(m, a, lt, bi, g, R2, flushes, sweep);
    bool listed = flushes == 0;
    // Everything after the staging: lists or re-tested sweeps, the Newton
    // iteration, the outputs.
    int redo = 0;
    auto density_sweeps = [&]() {
        // Neighbour lists, per i-slot in staged order: the staged candidates
        // within R of the slot's particle (fixed h: within its support, which
        // may reach R itself).
        constexpr int NENT = WaveMem<T, CAP, 1>::NENT;
        const int capl = NENT / c;
        int lcnt = 0;  // lane l < c: entries of i-slot l
        if (listed) {
            const T RL2 = max(R2, H2);
            for (int b = 0; b < ns; b += WAVE) {
                const int k = b + lane;
                const bool have = k < ns;
                const V4<T> sj = m.s[0][have ? k : 0];
                for (int l = 0; l < c; ++l) {
                    const int ll = l * S;  // the slot's first stream
                    const T px = lane_val(pi.x, ll), py = lane_val(pi.y, ll), pz = lane_val(pi.z, ll);
                    const bool in = have && dist2_unfused(px - sj.x, py - sj.y, pz - sj.z) <
                                                lane_val(RL2, ll);
                    const unsigned long long mk = ballot(in);
                    const int at = lane_val(lcnt, l) + mbcnt(mk);
                    if (in && at < capl) m.ent[l * capl + at] = (uint16_t)k;
                    if (lane == l) lcnt += __popcll(mk);
                }
            }
            listed = ballot(lane < c && lcnt > capl) == 0ull;
            tested += (unsigned long long)ns;  // per i-particle
            wave_sync();
        }
        constexpr int U = 2;   // list entries of a stream in flight together
        constexpr int UF = 2;  // the same in the full sweep (two global loads each)
        if (listed) {
            // stream js of slot li takes entries js, js + S, ... of li's list
            const int nl = act ? __shfl(lcnt, q.li, WAVE) : 0;
            const int nmax = uniform(wave_max(nl));
            const uint16_t* el = &m.ent[q.li * capl];
            int evals = 0;
            int sweeps = 0;
            allow_pred = true;
            for (int round = 0; round < 2; ++round) {
                // light sweeps until every particle has converged, needs a
                // wider staged set, or took a small step
                for (;;) {
                    ++sweeps;
                    ++iters;
                    // sweep at h: n and its first two log-h derivatives only
                    T s0 = 0, s1 = 0, s2 = 0;
                    for (int t0 = 0; t0 < nmax; t0 += U * S) {
                        V4<T> sj[U];
                        bool ok[U];
    #pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int e = t0 + u * S + js;
                            ok[u] = e < nl;
                            sj[u] = m.s[0][ok[u] ? el[e] : 0];
                        }
    #pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const T r2 =
                                dist2_unfused(pi.x - sj[u].x, pi.y - sj[u].y, pi.z - sj[u].z);
                            if (ok[u] && r2 < H2) {
                                const T inv_r = r2 > (T)0 ? fast_rsqrt(r2) : (T)0;
                                const T qq = r2 * inv_r * invH;
                                T w, s1v, gq;
                                m4_terms(qq, H * inv_r, w, s1v, gq);
                                s0 += w;
                                s1 += s1v;
                                s2 += m4_q2w2(qq);
                            }
                        }
                    }
                    evals += nl;
                    newton(group_sum(s0, S), group_sum(s1, S), group_sum(s2, S));
                    if (ballot(!conv && !pend && !pred) == 0ull) break;
                    if (sweeps >= a.h_max_iter) break;
                    next_h();
                }
                next_h();  // a small step moved h (the others keep theirs)
                vi = a.vel4[i];
                // the full sums at the final h (partner data from global
                // memory, the loads of UF entries issued together)
                zero();
                for (int t0 = 0; t0 < nmax; t0 += UF * S) {
                    V4<T> sj[UF], pj[UF], vj[UF];
                    bool in[UF];
    #pragma unroll
                    for (int u = 0; u < UF; ++u) {
                        const int e = t0 + u * S + js;
                        const bool ok = e < nl;
                        sj[u] = m.s[0][ok ? el[e] : 0];
                        in[u] = ok && dist2_unfused(pi.x - sj[u].x, pi.y - sj[u].y,
                                                    pi.z - sj[u].z) < H2;
                    }
    #pragma unroll
                    for (int u = 0; u < UF; ++u) {
                        int j = in[u] ? as_int<T>(sj[u].w) : 0;
                        if (j < 0 || j >= a.n) j = 0;  // cannot happen with a valid list
                        pj[u] = a.pos4[j];
                        vj[u] = a.vel4[j];
                    }
    #pragma unroll
                    for (int u = 0; u < UF; ++u)
                        if (in[u]) body(sj[u], pj[u], vj[u]);
                }
                evals += nl;
                if (round == 1) break;
                // a particle whose last step was small checks the stop
                // criterion on the full sums; one that fails it iterates on
                // from them (no small-step exits then) and the full sweep is
                // repeated (identical sums for the others)
                const T G = group_sum(S0, S), G1 = group_sum(S1, S), G2 = group_sum(S2, S);
                bool again = false;
                if (pred) {
                    pred = false;
                    if (fabs(G - Tt) <= a.h_tol * Tt) conv = true;
                    else again = true;
                }
                if (ballot(again) == 0ull || sweeps >= a.h_max_iter) break;
                allow_pred = false;
                if (again) newton(G, G1, G2);
                next_h();
            }
            // tests: the list pass plus every list evaluation
            tested_lane += lead ? (unsigned long long)evals : 0ull;
        } else {
            vi = a.vel4[i];
            sweep(ns);
            const bool cached = flushes == 0;
            T Rc = R;  // radius of the staged set
            for (int sweeps = 1; sweeps <= a.h_max_iter; ++sweeps) {
                ++iters;
                newton(group_sum(S0, S), group_sum(S1, S), group_sum(S2, S));
                if (ballot(!conv && !pend) == 0ull) break;
                if (sweeps == a.h_max_iter) break;
                next_h();
                zero();
                // the staged set follows the sweep's largest support (the
                // bounding-box distance never exceeds a lane's distance): a
                // cached set is compacted in LDS when that support shrank and
                // staged again from the list when h grew past it (it fit at R, so
                // it fits at any smaller radius); a set that did not fit is
                // staged again every sweep
                const T Hs = wave_max(act ? H : (T)0) * ((T)1 + (T)4 * tiny);
                bool restage = !cached;
                T Rs = Hs < R ? Hs : R;
                if (cached) {
                    if (Hs > Rc) {
                        Rc = min(R, Hs * (T)1.05);
                        Rs = Rc;
                        restage = true;
                    } else if (Hs < (T)0.9 * Rc) {
                        Rc = Hs * (T)1.05;
                        ns = compact_staged(m, ns, g, Rc * Rc);
                    }
                }
                if (restage) {
                    int fl = 0;
                    ns = stage_tile<L_DENS, T, CAP>(m, a, lt, bi, g, Rs * Rs, fl, sweep);
                }
                sweep(ns);
            }
        }
        S0 = group_sum(S0, S);
        S1 = group_sum(S1, S);
        Sr = group_sum(Sr, S);
        Sdr = group_sum(Sdr, S);
        Dv = group_sum(Dv, S);
        Cx = group_sum(Cx, S);
        Cy = group_sum(Cy, S);
        Cz = group_sum(Cz, S);
        cnt = group_sum(cnt, S);
        const bool last = a.fixup == 2;
        if (pend && last) { failed = true; pend = false; }
        if (!conv && !pend && act) failed = true;
        // outputs (sorted order): h rho rho_dh wcount wcount_dh div cx cy cz f | nngb iters
        bool beyond = false;
        if (lead) {
            // reciprocals (the hardware's in FP32, within an ulp) instead of
            // divisions
            const T ih = step_rcp(h);
            const T iH = ih / eps;
            const T k3 = cnorm * iH * iH * iH;
            const T k5 = k3 * iH * iH;
            const T rho = k3 * Sr;
            const T irho = step_rcp(rho);
            const T drho = -k3 * Sdr * ih;
            const int64_t n = a.n;
            T* o = a.out;
            o[0 * n + i] = h;
            o[1 * n + i] = rho;
            o[2 * n + i] = drho;
            o[3 * n + i] = k3 * S0;
            o[4 * n + i] = -k3 * S1 * ih;
            o[5 * n + i] = -k5 * Dv * irho;
            o[6 * n + i] = k5 * Cx * irho;
            o[7 * n + i] = k5 * Cy * irho;
            o[8 * n + i] = k5 * Cz * irho;
            o[9 * n + i] = step_rcp((T)1 + h * drho * irho * ((T)1 / (T)3));
            a.iout[0 * n + i] = cnt - 1;
            a.iout[1 * n + i] = failed ? -iters : iters;
            a.hs[i] = pend ? -want : h;  // negated: pending, for the next pass
            if constexpr (SINGLE) {
                const T gm1 = a.gamma - (T)1;
                const T u = vi.w;
                const T fi = o[9 * n + i];
                a.dens4_out[i] = V4<T>{rho, fi, sqrt(a.gamma * gm1 * u), fi * gm1 * u / rho};
                // a support beyond the margin over the guess and beyond the
                // box's smallest list radius
                const T rmin = (T)__uint_as_float(a.boxph[(BOX_STRIDE + 1) * a.n_box + tl.box]);
                const T hh = h * ((T)1 + (T)1e-5);
                beyond = !fixed && !pend &&
                         (failed || (hh > a.hguess[i] * a.dmargin && eps * hh > rmin));
            }
        }
        const unsigned long long pmask = ballot(pend);
        const unsigned long long fmask = ballot(failed && js == 0);
        T wmax = 0;
        if (pmask) wmax = wave_max(pend ? want : (T)0);
        if (lane == 0) {
            if (pmask) {
                T Rn = eps * wmax * (T)1.0625;
                if (!(Rn < Rcap)) Rn = Rcap;
                a.trad[t] = (float)Rn;
                a.tflag[t] = 1;
            } else {
                a.tflag[t] = 0;
            }
            if (fmask) latch(a.cnt, R >= Rcap ? (SWSPH_ST_REACH | SWSPH_ST_NEWTON) : SWSPH_ST_NEWTON);
        }
        ws.restages += pmask ? 1ull : 0ull;
        ws.tested += tested * (unsigned long long)nsel;
        // per-lane statistics, reduced over the wavefront once per launch
        ws.lane_tested += tested_lane;
        ws.lane_inside += lead ? (unsigned long long)cnt : 0ull;
        ws.lane_smax = max(ws.lane_smax, iters);
        ws.sweeps += (unsigned long long)(iters - iters0);
        ws.failed += (unsigned long long)__popcll(fmask);
        if constexpr (SINGLE) redo = (pmask != 0ull ? 1 : 0) | (ballot(beyond) != 0ull ? 2 : 0);
    };
    density_sweeps();
    ws.listed += listed ? 1ull : 0ull;
    return redo;
}

// ------------------------------------------------- gradient and force tile
// One staging and one pass of distance tests serve both loops: the force
// hits (r < max(H_i, H_j), Eq. 17-18) contain the gradient pairs (r < H_i,
// Eq. 10-11, 13), whose terms are added where r < H_i.  The gradient loop's
// outputs do not feed the force loop (alpha is constant, and the pairwise
// signal speed enters Eq. 9), so nothing orders the two.

// SINGLE: stage with radius Rown instead of the task build's (the
// single-launch step's lists were built with a larger one).
template <typename T, int CAP, bool SINGLE = false>
__device__ __forceinline__ void force_tile(WaveMem<T, CAP, 4>& m, const KArgs<T>& a, int t,
                                           WaveStats& ws, float Rown = 0.f) {
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
    const T h = a.hs[i];
    const TileGeom g = geom_of(tl);
    const T eps = a.eps;
    const T H = mul_unfused(eps, h);
    const T H2 = act ? mul_unfused(H, H) : (T)-1;
    const T invH = (T)1 / H;
    const T R = (T)(SINGLE ? Rown : a.trad[t]);
    const T cn = (T)(8.0 / PI_D);
    const T kgi = cn * invH * invH * invH * invH;
    const T rhoi = di.x, fi = di.y, ci = di.z, Ai = di.w;
    const bool visc = (a.flags & SWSPH_NO_VISC) == 0;
    const T alpha = a.alpha, beta = a.beta;
    T ax = 0, ay = 0, az = 0, du = 0;
    int nint = 0;
    const T ui = vi.w;
    T vsig = (T)2 * ci, lap = 0;  // gradient loop
    int ginside = 0;
    unsigned long long tested = 0;
    // hits: every j (self included) with r < max(H_i, H_j), counted in the
    // body (nint = hits - 1: the self pair is staged exactly once).  The self
    // pair and coincident pairs (r = 0) add nothing: 1/r is taken as 0 there,
    // which zeroes their a and du/dt terms, and the gradient terms skip them.
    int hits = 0;
    auto test = [&](int k, bool ok) {
        const V4<T> sj = m.s[0][k];
        const T r2 = dist2_unfused(pi.x - sj.x, pi.y - sj.y, pi.z - sj.z);
        // no short-circuit: the whole 4-vector is read up front
        return ok & act & (r2 < max_sq(H2, sj.w));
    };
    auto body = [&](int k) {
        const V4<T> sj = m.s[0][k];
        const T dx = pi.x - sj.x, dy = pi.y - sj.y, dz = pi.z - sj.z;
        const T r2 = dist2_unfused(dx, dy, dz);
        const T H2j = sj.w;
        const V4<T> vj = m.s[1][k];
        const V4<T> cj = m.s[2][k];  // (m_j, m_j A_j, m_j f_j, 1/H_j)
        const V4<T> ej = m.s[3][k];  // (rho_j, 8/(pi H_j^4), u_j, m_j / rho_j)
        const T rhoj = ej.x;
        ++hits;
        const bool pos = r2 > (T)0;
        const T inv_r = pos ? fast_rsqrt(r2) : (T)0;
        const T r = r2 * inv_r;
        const bool gin = pos & (r2 < H2);  // inside the support of i: a gradient pair
        const T gi = gin ? kgi * m4_dw(r * invH) : (T)0;
        const T ihj = cj.w;
        const T gj = r2 < H2j ? ej.y * m4_dw(r * ihj) : (T)0;
        const T vr = (vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz;
        const T vdote = vr * inv_r;
        const T mu = vdote < (T)0 ? vdote : (T)0;
        const T vs = ci + vj.w - beta * mu;
        T nu = 0;
        if (visc) nu = -alpha * mu * vs * fast_rcp(rhoi + rhoj);
        // gradient loop: signal speed and the Laplacian of u
        const T q = r * invH;
        const T t1 = (T)1 - q;
        const T gq = q < (T)0.5 ? (T)18 * q - (T)12 : (T)-6 * t1 * t1 * (H * inv_r);
        vsig = gin && vs > vsig ? vs : vsig;
        lap += gin ? ej.w * (ui - ej.z) * gq : (T)0;
        ginside += gin ? 1 : 0;
        const T mfg = cj.x * fi * gi + cj.z * gj;
        const T sa = cj.x * Ai * gi + cj.y * gj + (T)0.5 * nu * mfg;
        const T sr = sa * inv_r;
        ax -= sr * dx;
        ay -= sr * dy;
        az -= sr * dz;
        du += vdote * (cj.x * Ai * gi + (T)0.25 * nu * mfg);
    };
    auto sweep = [&](int ns) {
        pair_loop(m, ns, js, S, test, body);
        tested += (unsigned long long)ns;
    };
    int flushes = 0;
    const int ns = stage_tile<L_FORCE, T, CAP>(m, a, t, bi, g, R * R, flushes, sweep);
    sweep(ns);
    ax = stream_sum(ax, q);
    ay = stream_sum(ay, q);
    az = stream_sum(az, q);
    du = stream_sum(du, q);
    nint = stream_sum(hits, q) - 1;
    vsig = stream_max(vsig, q);
    lap = stream_sum(lap, q);
    ginside = stream_sum(ginside, q);
    if (lead) {
        a.out[0 * a.n + i] = ax;
        a.out[1 * a.n + i] = ay;
        a.out[2 * a.n + i] = az;
        a.out[3 * a.n + i] = du;
        a.iout[i] = nint;
        const T k5 = cn * invH * invH * invH * invH * invH;
        a.gout[0 * a.n + i] = vsig;
        a.gout[1 * a.n + i] = (T)2 * k5 * lap;
    }
    ws.inside += (unsigned long long)wave_sum(lead ? nint : 0);
    ws.inside_g += (unsigned long long)wave_sum(lead ? ginside : 0);
    ws.tested += tested * (unsigned long long)tl.count;
}

// ------------------------------------------- loops with time-dependent switches
// The SPHENIX-type switches (Sec. 2.1.3 Eq. 12-16, Sec. 2.1.4 Eq. 19-24) need
// the gradient loop's results before the force loop: the viscosity
// coefficient alpha_V is updated after the density loop, the gradient loop
// gives v_sig, the Laplacian of u and the largest alpha_V over each
// particle's support, the conduction coefficient alpha_c is updated from
// them, and only then runs the force loop with alpha_ij = mean(alpha_V)
// mean(B) and artificial conduction.  So the two loops run as two kernels
// over the same (force) task lists.  aux4 holds (alpha_V, B, alpha_c, 0) per
// binned particle.

// Gradient loop (r < H_i): v_sig, the Laplacian of u, and max alpha_V over
// the support, the particle itself and coincident neighbours included.
template <typename T, int CAP>
__device__ void grad_sw_tile(WaveMem<T, CAP, 3>& m, const KArgs<T>& a, int t, WaveStats& ws) {
    Tile tl = a.tiles[t];
    tl.begin = uniform(tl.begin);
    tl.count = uniform(tl.count);
    tl.box = uniform(tl.box);
    if (tl.count <= 0) return;
    const LaneMap q = lane_map(tl.count);
    const int js = q.js, S = q.S;
    const bool act = q.used();
    const bool lead = act && js == 0;
    const int i = tl.begin + (act ? q.li : 0);
    const BoxInfo bi = a.boxtab[tl.box];
    const V4<T> pi = a.pos4[i];
    const V4<T> vi = a.vel4[i];
    const V4<T> di = a.dens4[i];  // (rho, f, c, A)
    const T h = a.hs[i];
    const TileGeom g = geom_of(tl);
    const T H = mul_unfused(a.eps, h);
    const T H2 = act ? mul_unfused(H, H) : (T)-1;
    const T invH = (T)1 / H;
    const T R = (T)a.trad[t];
    const T cn = (T)(8.0 / PI_D);
    const T ci = di.z, ui = vi.w;
    T vsig = (T)2 * ci, lap = 0, avmax = a.aux4[i].x;
    int inside = 0;
    unsigned long long tested = 0;
    auto test = [&](int k, bool ok) {
        const V4<T> sj = m.s[0][k];
        return ok & (dist2_unfused(pi.x - sj.x, pi.y - sj.y, pi.z - sj.z) < H2);
    };
    auto body = [&](int k) {
        const V4<T> sj = m.s[0][k];   // (x, y, z, m_j / rho_j)
        const V4<T> vj = m.s[1][k];   // (v, c_j)
        const V4<T> wj = m.s[2][k];   // (u_j, alpha_V,j)
        avmax = wj.y > avmax ? wj.y : avmax;
        const T dx = pi.x - sj.x, dy = pi.y - sj.y, dz = pi.z - sj.z;
        const T r2 = dist2_unfused(dx, dy, dz);
        if (r2 > (T)0) {
            const T inv_r = fast_rsqrt(r2);
            const T r = r2 * inv_r;
            const T vr = (vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz;
            const T vdote = vr * inv_r;
            const T mu = vdote < (T)0 ? vdote : (T)0;
            const T vs = ci + vj.w - a.beta * mu;
            vsig = vs > vsig ? vs : vsig;
            const T qq = r * invH;
            const T t1 = (T)1 - qq;
            const T gq = qq < (T)0.5 ? (T)18 * qq - (T)12 : (T)-6 * t1 * t1 * (H * inv_r);
            lap += sj.w * (ui - wj.x) * gq;
            ++inside;
        }
    };
    auto sweep = [&](int ns) {
        pair_loop(m, ns, js, S, test, body);
        tested += (unsigned long long)ns;
    };
    int flushes = 0;
    const int ns = stage_tile<L_GSW, T, CAP>(m, a, t, bi, g, R * R, flushes, sweep);
    sweep(ns);
    vsig = stream_max(vsig, q);
    avmax = stream_max(avmax, q);
    lap = stream_sum(lap, q);
    inside = stream_sum(inside, q);
    if (lead) {
        const T k5 = cn * invH * invH * invH * invH * invH;
        a.gout[0 * a.n + i] = vsig;
        a.gout[1 * a.n + i] = (T)2 * k5 * lap;
        a.gout[2 * a.n + i] = avmax;
    }
    ws.inside += (unsigned long long)wave_sum(lead ? inside : 0);
    ws.tested += tested * (unsigned long long)tl.count;
}

// Force loop with alpha_ij = (alpha_V,i + alpha_V,j)/2 (B_i + B_j)/2 in the
// viscosity (Eq. 9, 16) and artificial conduction in du/dt (Eq. 19-20, 22).
template <typename T, int CAP>
__device__ void force_sw_tile(WaveMem<T, CAP, 5>& m, const KArgs<T>& a, int t, WaveStats& ws) {
    Tile tl = a.tiles[t];
    tl.begin = uniform(tl.begin);
    tl.count = uniform(tl.count);
    tl.box = uniform(tl.box);
    if (tl.count <= 0) return;
    const LaneMap q = lane_map(tl.count);
    const int js = q.js, S = q.S;
    const bool act = q.used();
    const bool lead = act && js == 0;
    const int i = tl.begin + (act ? q.li : 0);
    const BoxInfo bi = a.boxtab[tl.box];
    const V4<T> pi = a.pos4[i];
    const V4<T> vi = a.vel4[i];
    const V4<T> di = a.dens4[i];  // (rho, f, c, A)
    const V4<T> swi = a.aux4[i];  // (alpha_V, B, alpha_c, 0)
    const T h = a.hs[i];
    const TileGeom g = geom_of(tl);
    const T eps = a.eps;
    const T H = mul_unfused(eps, h);
    const T H2 = act ? mul_unfused(H, H) : (T)-1;
    const T invH = (T)1 / H;
    const T R = (T)a.trad[t];
    const T cn = (T)(8.0 / PI_D);
    const T kgi = cn * invH * invH * invH * invH;
    const T rhoi = di.x, fi = di.y, ci = di.z, Ai = di.w, ui = vi.w;
    const T Pi = (a.gamma - (T)1) * rhoi * ui;
    const bool visc = (a.flags & SWSPH_NO_VISC) == 0;
    T ax = 0, ay = 0, az = 0, du = 0;
    unsigned long long tested = 0;
    int hits = 0;
    auto test = [&](int k, bool ok) {
        const V4<T> sj = m.s[0][k];
        const T r2 = dist2_unfused(pi.x - sj.x, pi.y - sj.y, pi.z - sj.z);
        // no short-circuit: the whole 4-vector is read up front, so the
        // reads of consecutive tests issue together
        const bool in = ok & act & ((r2 < H2) | (r2 < sj.w));
        hits += in ? 1 : 0;
        return in & (r2 > (T)0);
    };
    auto body = [&](int k) {
        const V4<T> sj = m.s[0][k];
        const T dx = pi.x - sj.x, dy = pi.y - sj.y, dz = pi.z - sj.z;
        const T r2 = dist2_unfused(dx, dy, dz);
        const V4<T> vj = m.s[1][k];  // (v, c_j)
        const V4<T> cj = m.s[2][k];  // (m_j, m_j A_j, m_j f_j, 1/H_j)
        const V4<T> ej = m.s[3][k];  // (rho_j, P_j, u_j, 0)
        const V4<T> wj = m.s[4][k];  // (alpha_V,j, B_j, alpha_c,j, 0)
        const T rhoj = ej.x;
        const T inv_r = fast_rsqrt(r2);
        const T r = r2 * inv_r;
        const T gi = r2 < H2 ? kgi * m4_dw(r * invH) : (T)0;
        const T ihj = cj.w;
        const T gj = r2 < sj.w ? cn * ihj * ihj * ihj * ihj * m4_dw(r * ihj) : (T)0;
        const T vr = (vi.x - vj.x) * dx + (vi.y - vj.y) * dy + (vi.z - vj.z) * dz;
        const T vdote = vr * inv_r;
        const T mu = vdote < (T)0 ? vdote : (T)0;
        const T vs = ci + vj.w - a.beta * mu;
        const T irs = fast_rcp(rhoi + rhoj);
        T nu = 0;
        if (visc) {
            const T aij = (T)0.25 * (swi.x + wj.x) * (swi.y + wj.y);
            nu = -aij * mu * vs * irs;
        }
        const T mfg = cj.x * fi * gi + cj.z * gj;
        const T sa = cj.x * Ai * gi + cj.y * gj + (T)0.5 * nu * mfg;
        const T sr = sa * inv_r;
        ax -= sr * dx;
        ay -= sr * dy;
        az -= sr * dz;
        du += vdote * (cj.x * Ai * gi + (T)0.25 * nu * mfg);
        // artificial conduction
        const T Pj = ej.y;
        const T psum = Pi + Pj;
        const T acij = psum > (T)0 ? (Pi * swi.z + Pj * wj.z) * fast_rcp(psum) : (T)0;
        const T vc = fabs(vdote) + sqrt((T)2 * fabs(Pi - Pj) * irs);
        du += acij * vc * (ui - ej.z) * mfg * irs;
    };
    auto sweep = [&](int ns) {
        pair_loop(m, ns, js, S, test, body);
        tested += (unsigned long long)ns;
    };
    int flushes = 0;
    const int ns = stage_tile<L_FSW, T, CAP>(m, a, t, bi, g, R * R, flushes, sweep);
    sweep(ns);
    ax = stream_sum(ax, q);
    ay = stream_sum(ay, q);
    az = stream_sum(az, q);
    du = stream_sum(du, q);
    const int nint = stream_sum(hits, q) - 1;
    if (lead) {
        a.out[0 * a.n + i] = ax;
        a.out[1 * a.n + i] = ay;
        a.out[2 * a.n + i] = az;
        a.out[3 * a.n + i] = du;
        a.iout[i] = nint;
    }
    ws.inside += (unsigned long long)wave_sum(lead ? nint : 0);
    ws.tested += tested * (unsigned long long)tl.count;
}

// ----------------------------------------------------------------- drivers

template <int LK, typename T, int CAP>
__device__ __forceinline__ void run_tile(char* wm, const KArgs<T>& a, int t, WaveStats& ws) {
    if (LK == L_DENS) density_tile<T, CAP>(*(WaveMem<T, CAP, 1>*)wm, a, t, ws);
    else if (LK == L_GSW) grad_sw_tile<T, CAP>(*(WaveMem<T, CAP, 3>*)wm, a, t, ws);
    else if (LK == L_FSW) force_sw_tile<T, CAP>(*(WaveMem<T, CAP, 5>*)wm, a, t, ws);
    else force_tile<T, CAP>(*(WaveMem<T, CAP, 4>*)wm, a, t, ws);
}

// Register budgets matching what LDS allows (FP32): three wavefronts per
// SIMD for the density kernel (its Newton accumulators would otherwise take
// it just past the 168-register step), four for the gradient/force kernel,
// three for the two loops with switches.
template <int LK>
constexpr int loop_stats_index() {
    return LK == L_DENS ? LOOP_DENSITY : (LK == L_GSW ? LOOP_GRADIENT : LOOP_FORCE);
}
template <int LK, typename T, int CAP>
__global__ void __launch_bounds__(WPB * WAVE)
SWSPH_WAVES_PER_EU(sizeof(T) != 4 ? 1 : (LK == L_FORCE ? 4 : 3))
k_loop(KArgs<T> a, int mode) {
    SWSPH_DYN_SHARED char smem[];
    constexpr size_t WMS = sizeof(WaveMem<T, CAP, LoopNV<LK>::NV>);
    const int wave = threadIdx.x / WAVE;
    char* wm = smem + wave * WMS;
    WaveStats ws;
    for_each_task(a, mode, [&](int t) { run_tile<LK, T, CAP>(wm, a, t, ws); });
    ws.flush(a.cnt, loop_stats_index<LK>(), LK == L_FORCE);
}

int device_cu_count() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 0;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

template <int LK, typename T, int CAP>
static int launch_loop_cap(KArgs<T> a, int mode, int queue_slot, hipStream_t s) {
    return launch_with<LK, T, CAP>(k_loop<LK, T, CAP>, a, mode, queue_slot, s);
}

// Largest staging capacity <= lds_cap whose workgroup fits in the LDS
// (1024 only for the density loop's fix-up passes).
template <int LK, typename T>
static int launch_loop(KArgs<T> a, int mode, int lds_cap, int queue_slot, hipStream_t s) {
    if constexpr (LK == L_DENS && fits<LK, T, 1024>())
        if (lds_cap >= 1024) return launch_loop_cap<LK, T, 1024>(a, mode, queue_slot, s);
    if (lds_cap >= 512 && fits<LK, T, 512>()) return launch_loop_cap<LK, T, 512>(a, mode, queue_slot, s);
    if (lds_cap >= 256 && fits<LK, T, 256>()) return launch_loop_cap<LK, T, 256>(a, mode, queue_slot, s);
    static_assert(fits<LK, T, 128>(), "staging buffer does not fit");
    return launch_loop_cap<LK, T, 128>(a, mode, queue_slot, s);
}

// Indices of the tiles flagged for a density fix-up (any order: tiles are
// independent).  Each wavefront owns FIX_RUNS consecutive runs of 64 tiles:
// it counts their flags, takes its space with one atomic (only if any are
// set) and writes them -- flagged tiles are few and scattered, so one atomic
// per 64 tiles left hundreds of wavefronts queueing on the same counter.
constexpr int FIX_RUNS = 16;
__global__ void k_fix_list(const int32_t* __restrict__ tflag,
                           const unsigned long long* __restrict__ ntiles,
                           Counters* __restrict__ cnt, int32_t* __restrict__ list) {
    const int64_t nt = (int64_t)*ntiles;
    const int lane = lane_id();
    const int64_t span = (int64_t)FIX_RUNS * WAVE;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    for (int64_t base = w * span; base < nt; base += nw * span) {
        int tot = 0;
        for (int r = 0; r < FIX_RUNS; ++r) {
            const int64_t t = base + (int64_t)r * WAVE + lane;
            tot += __popcll(ballot(t < nt && tflag[t] != 0));
        }
        if (tot == 0) continue;
        int at = 0;
        if (lane == 0) at = (int)atomicAdd(&cnt->n_fix, (unsigned long long)tot);
        at = __shfl(at, 0, WAVE);
        for (int r = 0; r < FIX_RUNS; ++r) {
            const int64_t t = base + (int64_t)r * WAVE + lane;
            const bool f = t < nt && tflag[t] != 0;
            const unsigned long long m = ballot(f);
            if (f) list[at + mbcnt(m)] = (int32_t)t;
            at += __popcll(m);
        }
    }
}

// Density fix-up passes over the tiles a first pass flagged (b.tflag, their
// wider radii in b.trad): each builds their lists and reruns them (any
// order); the last latches failures.
constexpr int DENS_FIXUPS = 3;
template <typename T>
static int density_fixups(const BinPtrs& b, const Scheme& sc, KArgs<T> a, int mode,
                          hipStream_t s) {
    a.order = b.tmpidx;
    a.ntask = &b.cnt->n_fix;
    a.xcd_split = 0;
    a.parent = nullptr;
    a.boxph = nullptr;
    int r = 0;
    for (int pass = 1; pass <= DENS_FIXUPS && !r; ++pass) {
        launch_fill_u32(&b.cnt->n_fix, 2, 0u, s);
        hipLaunchKernelGGL(k_fix_list, dim3(wave_grid((b.tile_cap + FIX_RUNS - 1) / FIX_RUNS, 4)),
                           dim3(256), 0, s,
                           (const int32_t*)b.tflag, (const unsigned long long*)b.ntiles, b.cnt,
                           b.tmpidx);
        launch_tasks<T>(b, sc, 0, true, s);
        a.fixup = pass == DENS_FIXUPS ? 2 : 1;
        timer_begin(sc.timer, 0, s);
        // fix-up tiles are few and their lists long: the largest staging
        // buffer keeps them in LDS across their sweeps
        r = launch_loop<L_DENS, T>(a, mode == MODE_PER_TASK ? MODE_FLAT : mode, 1024, 0, s);
        timer_end(sc.timer, 0, s);
    }
    return r;
}

// Density: the first pass, then the fix-up passes for tiles whose Newton
// iteration needed a wider task list.
template <typename T>
int launch_density(const BinPtrs& bin, const Scheme& sc, int mode, int lds_cap, hipStream_t s) {
    const BinPtrs b = density_view(bin);
    KArgs<T> a = make_args<T>(b, sc);
    a.out = (T*)b.d_out;
    a.iout = b.d_int;
    if (bin.tile_d < bin.tile) {
        // one list per gradient/force tile, at the margin over its largest
        // guessed support: its density tiles stage from it with their own
        // radius (each gets exactly the list of its own search, in order)
        launch_tasks<T>(bin, sc, 0, false, s);
        a.parent = bin.dparent;
        if (sc.order == 0) launch_order(b, s);
    } else {
        launch_tasks<T>(b, sc, 0, false, s);
    }
    timer_begin(sc.timer, 0, s);
    int r = launch_loop<L_DENS, T>(a, mode, lds_cap, 0, s);
    timer_end(sc.timer, 0, s);
    if (r || (sc.flags & SWSPH_FIXED_H)) return r;
    return density_fixups<T>(b, sc, a, mode, s);
}
// Task lists of the joint gradient/force loop: the force list (support
// max(H_i, H_j)) contains every pair the gradient loop needs (support H_i).
template <typename T>
void launch_gf_tasks(const BinPtrs& b, const Scheme& sc, hipStream_t s) {
    launch_hmax_pyramid<T>(b, sc, s);
    launch_tasks<T>(b, sc, 2, false, s);
}
template <typename T>
int launch_force(const BinPtrs& b, const Scheme& sc, int mode, int lds_cap, hipStream_t s) {
    KArgs<T> a = make_args<T>(b, sc);
    // one tile per queue pop (measured faster than two for this loop on a
    // clustered set; the density loop is faster with two per pop)
    a.qchunk = 1;
    a.out = (T*)b.f_out;
    a.gout = (T*)b.g_out;
    a.iout = b.f_int;
    timer_begin(sc.timer, 2, s);
    const int r = launch_loop<L_FORCE, T>(a, mode, lds_cap, 2, s);
    timer_end(sc.timer, 2, s);
    return r;
}

template int launch_density<float>(const BinPtrs&, const Scheme&, int, int, hipStream_t);
template int launch_density<double>(const BinPtrs&, const Scheme&, int, int, hipStream_t);
template void launch_gf_tasks<float>(const BinPtrs&, const Scheme&, hipStream_t);
template void launch_gf_tasks<double>(const BinPtrs&, const Scheme&, hipStream_t);
template int launch_force<float>(const BinPtrs&, const Scheme&, int, int, hipStream_t);
template int launch_force<double>(const BinPtrs&, const Scheme&, int, int, hipStream_t);

// ------------------------------------------------------ single launch
// Every box's density, gradient and force tiles in one persistent launch
// (Sec. 4: one kernel for many small, uneven tasks instead of a launch per
// task or per loop).  Each of the queue's XCD segments holds its share of
// the density tiles, then its share of the gradient/force tiles, both box
// by box.  A gradient/force tile first waits until its box's phase word
// counts all of the box's density tiles as done.  Density tiles wait for
// nothing, and a wavefront reaches a segment's gradient/force tiles only
// after every density tile of that segment has been popped; each segment is
// worked on by the wavefronts of its own XCD from the start, so every density
// tile waited for gets done (the grid never exceeds the co-resident
// workgroups either).  The wait is capped: a timeout latches LOOPCAP and
// leaves the box to the redo path.  The
// gradient/force lists were built before the launch at the density margin
// over the guessed supports; a tile runs on them when its box's h all ended
// within that margin (its density tiles set the redo bit otherwise) and its
// own radius at the final h fits its list's; the rest is redone afterwards.
constexpr int BOX_SPIN_MAX = 1 << 16;  // polls about 2 us apart: 0.1 s at most

// Density tiles of every box (the totals the phase words count up to):
// tiles come box by box, so each box's are a range found by binary search.
__global__ void k_box_tiles(const Tile* __restrict__ tiles_d, const unsigned long long* __restrict__ ntd,
                            int32_t n_box, uint32_t* __restrict__ total) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_box) return;
    const int64_t nt = (int64_t)*ntd;
    auto first = [&](int box) {  // first tile of a box >= box
        int64_t lo = 0, hi = nt;
        for (int it = 0; it < 64 && lo < hi; ++it) {
            const int64_t mid = (lo + hi) / 2;
            if (tiles_d[mid].box < box) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    total[b] = (uint32_t)(first(b + 1) - first(b));
}

// Smallest task-list radius of every box's gradient/force tiles (positive
// floats order as their bit patterns).
__global__ void k_box_rmin(const Tile* __restrict__ tiles, const unsigned long long* __restrict__ ntiles,
                           const float* __restrict__ trad, int32_t n_box, uint32_t* __restrict__ rmin) {
    const int64_t nt = (int64_t)*ntiles;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += nth) {
        int box = -1;
        float r = 3.0e38f;
        if (t < nt) {
            const Tile tl = tiles[t];
            if (tl.count > 0 && tl.box >= 0 && tl.box < n_box && trad[t] > 0.f) {
                box = tl.box;
                r = trad[t];
            }
        }
        // consecutive tiles mostly share a box: one atomic per wavefront then
        const int b0 = __shfl(box, 0, WAVE);
        if (ballot(box != b0) == 0ull) {
            const float m = wave_min(r);
            if (lane_id() == 0 && b0 >= 0) atomicMin(&rmin[b0], __float_as_uint(m));
        } else if (box >= 0) {
            atomicMin(&rmin[box], __float_as_uint(r));
        }
    }
}

// The launch's queue, cut (as the queue cuts any list) into NXCD segments
// [B_x, B_x+1), B_x = nt x / NXCD: segment x holds density tiles D_x ..
// D_x+1 - 1, D_x = B_x nd / nt, then gradient/force tiles (as nd + t) from
// B_x - D_x on -- both counts rise with x, so the lists stay in their order,
// box by box, and every segment has its density tiles first.
__global__ void k_single_order(const int32_t* __restrict__ order_d,
                               const unsigned long long* __restrict__ ntd,
                               const int32_t* __restrict__ order_f,
                               const unsigned long long* __restrict__ ntf,
                               int32_t* __restrict__ items, unsigned long long* __restrict__ nitems) {
    const int64_t nd = (int64_t)*ntd, nf = (int64_t)*ntf, nt = nd + nf;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    const int64_t k0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k0 == 0) *nitems = (unsigned long long)nt;
    for (int64_t k = k0; k < nt; k += nth) {
        int x = 0;
        while (x + 1 < NXCD && nt * (x + 1) / NXCD <= k) ++x;
        const int64_t bx = nt * x / NXCD, bx1 = nt * (x + 1) / NXCD;
        const int64_t dx = bx * nd / nt, dx1 = bx1 * nd / nt;
        const int64_t j = k - bx;
        items[k] = j < dx1 - dx ? order_d[dx + j]
                                : (int32_t)(nd + order_f[(bx - dx) + (j - (dx1 - dx))]);
    }
}

// ready: the box this wavefront last found complete (no second wait or
// acquire for its further tiles), or READY_ALL once every density tile of
// every box is done and acquired (one acquire for the rest of the launch).
constexpr int READY_ALL = -2;

// Word counting every box's density tiles done (its own cache line).
__device__ __forceinline__ int64_t box_all_word(int32_t n_box) {
    return ((int64_t)(BOX_STRIDE + 2) * n_box + BOX_STRIDE - 1) / BOX_STRIDE * BOX_STRIDE;
}

template <typename T, int CAP>
__device__ __forceinline__ void single_force_tile(WaveMem<T, CAP, 4>& m, const KArgs<T>& a, int t,
                                                  WaveStats& ws, int& ready, int64_t nd) {
    const Tile tl = a.tiles[t];
    const int count = uniform(tl.count), box = uniform(tl.box);
    if (count <= 0) return;
    const int lane = lane_id();
    if (ready != READY_ALL) {
        int all = 0;
        if (lane == 0)
            all = (int64_t)__hip_atomic_load(&a.boxph[box_all_word(a.n_box)], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT) >= nd;
        if (__shfl(all, 0, WAVE)) {
            __threadfence();  // acquire every box's density results at once
            ready = READY_ALL;
        }
    }
    if (ready == READY_ALL) {
        if (a.boxph[box * BOX_STRIDE] & BOX_REDO) return;
    } else if (box != ready) {
    uint32_t w = BOX_REDO;
    if (lane == 0) {
        const uint32_t need = a.boxph[BOX_STRIDE * a.n_box + box];
        int it = 0;
        for (; it < BOX_SPIN_MAX; ++it) {
            const uint32_t v = __hip_atomic_load(&a.boxph[box * BOX_STRIDE], __ATOMIC_ACQUIRE,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            // a box already sent to the redo path needs no waiting
            if ((v & BOX_DONE) >= need || (v & BOX_REDO)) {
                w = v;
                break;
            }
            // poll gently: thousands of waiting wavefronts on a few words
            // would otherwise crowd the cache channel that holds them
            __builtin_amdgcn_s_sleep(64);
        }
        if (it == BOX_SPIN_MAX) {
            // cannot happen with the queue order above; the box is redone
            // (and later waits on it end at once)
            latch(a.cnt, SWSPH_ST_LOOPCAP);
            atomicOr(&a.boxph[box * BOX_STRIDE], BOX_REDO);
        }
    }
    w = (uint32_t)__shfl((int)w, 0, WAVE);
    // acquire: the box's density results (one cache invalidation per box
    // and wavefront: across XCDs this is costly)
    __threadfence();
    if (w & BOX_REDO) return;  // the redo path takes the whole box
    ready = box;
    } else if (a.boxph[box * BOX_STRIDE] & BOX_REDO) {
        return;
    }
    const int begin = uniform(tl.begin);
    const T hi = lane < count ? a.hs[begin + lane] : (T)0;
    const T hmax = wave_max(hi);
    // the radius a task build at the final h would give the tile
    const float L = (float)a.boxtab[box].L;
    const float R = (float)(a.eps * hmax * (T)(1 + 4e-7));
    if (!(R < 0.5f * L * (1.0f - 1e-6f)) || !(R <= a.trad[t]) || !(R > 0.f)) {
        if (lane == 0) a.fredo[t] = 1;
        return;
    }
    force_tile<T, CAP, true>(m, a, t, ws, R);
}

template <typename T, int CAPD, int CAPF>
__global__ void __launch_bounds__(WPB * WAVE) SWSPH_WAVES_PER_EU(sizeof(T) != 4 ? 1 : 3)
k_single(KArgs<T> ad, KArgs<T> af, KArgs<T> aq) {
    SWSPH_DYN_SHARED char smem[];
    constexpr size_t WMD = sizeof(WaveMem<T, CAPD, 1>), WMF = sizeof(WaveMem<T, CAPF, 4>);
    constexpr size_t WMS = WMD > WMF ? WMD : WMF;
    const int wave = threadIdx.x / WAVE;
    char* wm = smem + wave * WMS;
    const int64_t nd = (int64_t)*ad.ntask;
    WaveStats wsd, wsf;
    // density tiles done by this wavefront, not yet counted: box, count,
    // redo.  They are released together (one fence) when the box changes,
    // before the first gradient/force tile and at the end: a wavefront never
    // waits while it holds uncounted tiles, so every wait still ends.
    int sbox = -1, ready = -1;
    uint32_t scnt = 0;
    bool sredo = false;
    auto release = [&]() {
        if (sbox < 0) return;
        __threadfence();
        if (lane_id() == 0) {
            if (sredo) atomicOr(&ad.boxph[sbox * BOX_STRIDE], BOX_REDO);
            atomicAdd(&ad.boxph[sbox * BOX_STRIDE], scnt);
            atomicAdd(&ad.boxph[box_all_word(ad.n_box)], scnt);
        }
        sbox = -1;
        scnt = 0;
        sredo = false;
    };
    for_each_task(aq, MODE_QUEUE, [&](int k) {
        if (k < nd) {
            const Tile tl = ad.tiles[k];
            const int box = uniform(tl.box);
            if (box != sbox) release();
            sbox = box;
            auto& md = *(WaveMem<T, CAPD, 1>*)wm;
            int code = density_tile<T, CAPD, true>(md, ad, k, wsd);
            if (code == 1) {
                // an h needs a wider staged set: the tile's h (the converged
                // ones, and, negated, the wider guesses the others asked
                // for) are in hs; run it again at once when its
                // gradient/force tile's list covers the wider radius (the
                // fix-up path otherwise)
                const int count = uniform(tl.count), begin = uniform(tl.begin);
                const T hm = wave_max(lane_id() < count ? fabs(ad.hs[begin + lane_id()]) : (T)0);
                const float Rn = (float)(ad.eps * hm * (T)1.0625);
                const float Rp = af.trad[uniform(ad.parent[k])];
                if (Rn <= Rp) code = density_tile<T, CAPD, true>(md, ad, k, wsd, Rp);
            }
            sredo = sredo || code != 0;
            ++scnt;
        } else {
            release();
            single_force_tile<T, CAPF>(*(WaveMem<T, CAPF, 4>*)wm, af, (int)(k - nd), wsf, ready,
                                       nd);
        }
    });
    release();
    wsd.flush(ad.cnt, LOOP_DENSITY, false);
    wsf.flush(af.cnt, LOOP_FORCE, true);
}

// Gradient/force tiles the single launch left: flagged by the tile, or in a
// box with the redo bit.  fredo[t] becomes the flag, the list goes to tmpidx.
__global__ void k_redo_list(const Tile* __restrict__ tiles, const unsigned long long* __restrict__ ntiles,
                            const uint32_t* __restrict__ boxph, int32_t n_box,
                            int32_t* __restrict__ fredo, Counters* __restrict__ cnt,
                            int32_t* __restrict__ list) {
    const int64_t nt = (int64_t)*ntiles;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < nt; base += nth) {
        const int64_t t = base + threadIdx.x;
        bool f = false;
        if (t < nt) {
            const int b = tiles[t].box;
            f = fredo[t] != 0 || (b >= 0 && b < n_box && (boxph[b * BOX_STRIDE] & BOX_REDO) != 0u);
            fredo[t] = f ? 1 : 0;
        }
        const unsigned long long m = ballot(f);
        int at = 0;
        if (lane_id() == 0 && m) {
            at = (int)atomicAdd(&cnt->n_fix, (unsigned long long)__popcll(m));
            atomicAdd(&cnt->single_redo, (unsigned long long)__popcll(m));
        }
        at = __shfl(at, 0, WAVE);
        if (f) list[at + mbcnt(m)] = (int32_t)t;
    }
}

// (rho, f, c, A) of every binned particle from the binned density results.
template <typename T>
__global__ void k_dens4_binned(int64_t n, const T* __restrict__ dout,
                               const V4<T>* __restrict__ vel4, T gamma,
                               V4<T>* __restrict__ dens4) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const T rho = dout[1 * n + s], f = dout[9 * n + s], u = vel4[s].w;
    const T gm1 = gamma - (T)1;
    dens4[s] = V4<T>{rho, f, sqrt(gamma * gm1 * u), f * gm1 * u / rho};
}

template <typename T>
__global__ void k_copy_n(int64_t n, const T* __restrict__ in, T* __restrict__ out) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s < n) out[s] = in[s];
}

template <typename T, int CAPD, int CAPF>
static int launch_single_cap(const KArgs<T>& ad, const KArgs<T>& af, const KArgs<T>& aq,
                             hipStream_t s) {
    void (*kern)(KArgs<T>, KArgs<T>, KArgs<T>) = k_single<T, CAPD, CAPF>;
    constexpr size_t WMD = sizeof(WaveMem<T, CAPD, 1>), WMF = sizeof(WaveMem<T, CAPF, 4>);
    const size_t shm = (WMD > WMF ? WMD : WMF) * WPB;
    static bool attr_set = false;
    if (!attr_set) {
        if (hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm) != hipSuccess)
            return -1;
        attr_set = true;
    }
    launch_fill_u32(aq.queue, 2 * NXCD, 0u, s);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, WPB * WAVE, shm) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t blocks = (int64_t)per_cu * device_cu_count();
    const int64_t need = (aq.tile_cap + WPB - 1) / WPB;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(WPB * WAVE), shm, s, ad, af, aq);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_single(const BinPtrs& bin, const Scheme& sc, int lds_cap_d, int lds_cap,
                  hipStream_t s) {
    if (bin.n <= 0) return 0;
    const BinPtrs bd = density_view(bin);
    // gradient/force lists at the margin over the guessed supports; the
    // density tiles stage from them as from their parent's density list
    launch_hmax_pyramid<T>(bin, sc, s);
    launch_tasks<T>(bin, sc, 3, false, s);
    const int32_t nb = bin.n_box;
    const unsigned gn = (unsigned)((bin.n + 255) / 256);
    // the guesses, for the check of each h against them (the third gradient
    // output array is free in this step)
    T* hguess = (T*)bin.g_out + 2 * bin.n;
    hipLaunchKernelGGL(k_copy_n<T>, dim3(gn), dim3(256), 0, s, bin.n, (const T*)bin.hs, hguess);
    uint32_t* total = bin.boxph + (int64_t)BOX_STRIDE * nb;
    uint32_t* rmin = total + nb;
    launch_fill_u32(bin.boxph, (int64_t)BOX_STRIDE * nb, 0u, s);
    const int64_t all_word = ((int64_t)(BOX_STRIDE + 2) * nb + BOX_STRIDE - 1) / BOX_STRIDE * BOX_STRIDE;
    launch_fill_u32(bin.boxph + all_word, 1, 0u, s);
    launch_fill_u32(rmin, nb, 0x7f7fffffu, s);  // FLT_MAX
    launch_fill_u32(bin.fredo, bin.tile_cap, 0u, s);
    hipLaunchKernelGGL(k_box_tiles, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s,
                       (const Tile*)bd.tiles, (const unsigned long long*)bd.ntiles, nb, total);
    hipLaunchKernelGGL(k_box_rmin, dim3(wave_grid(bin.tile_cap, 4)), dim3(256), 0, s,
                       (const Tile*)bin.tiles, (const unsigned long long*)bin.ntiles,
                       (const float*)bin.trad, nb, rmin);
    hipLaunchKernelGGL(k_single_order, dim3(wave_grid(2 * bin.tile_cap, 4)), dim3(256), 0, s,
                       (const int32_t*)bd.order, (const unsigned long long*)bd.ntiles,
                       (const int32_t*)bin.order, (const unsigned long long*)bin.ntiles,
                       bin.forder, &bin.cnt->n_items);
    KArgs<T> ad = make_args<T>(bd, sc);
    ad.out = (T*)bd.d_out;
    ad.iout = bd.d_int;
    ad.parent = bin.dparent;
    ad.trad = bin.trad_d;  // fix-up radii: the lists' radii stay for the check above
    ad.dens4_out = (V4<T>*)bin.dens4;
    ad.hguess = hguess;
    if (!(sc.flags & SWSPH_FIXED_H)) ad.dmargin = (T)SINGLE_MARGIN;
    ad.boxph = bin.boxph;
    KArgs<T> af = make_args<T>(bin, sc);
    af.out = (T*)bin.f_out;
    af.gout = (T*)bin.g_out;
    af.iout = bin.f_int;
    af.boxph = bin.boxph;
    af.fredo = bin.fredo;
    KArgs<T> aq = ad;
    aq.order = bin.forder;
    aq.ntask = &bin.cnt->n_items;
    aq.tile_cap = 2 * bin.tile_cap;
    aq.xcd_split = 1;  // per XCD, density tiles first in each segment
    aq.qchunk = 4;
    aq.queue = bin.cnt->queue[1];
    int r;
    if constexpr (sizeof(T) == 4) {
        if (lds_cap_d >= 512) r = launch_single_cap<T, 512, 128>(ad, af, aq, s);
        else if (lds_cap_d >= 256) r = launch_single_cap<T, 256, 128>(ad, af, aq, s);
        else r = launch_single_cap<T, 128, 128>(ad, af, aq, s);
    } else {
        r = launch_single_cap<T, 128, 128>(ad, af, aq, s);
    }
    (void)lds_cap;
    if (r) return r;
    // what the launch left: density fix-ups (their radii in trad_d), then
    // the gradient/force tiles of boxes with the redo bit or flagged
    if (!(sc.flags & SWSPH_FIXED_H)) {
        BinPtrs bx = bd;
        bx.trad = bin.trad_d;
        r = density_fixups<T>(bx, sc, ad, MODE_QUEUE, s);
        if (r) return r;
        hipLaunchKernelGGL(k_dens4_binned<T>, dim3(gn), dim3(256), 0, s, bin.n,
                           (const T*)bin.d_out, (const V4<T>*)bin.vel4, (T)sc.gamma,
                           (V4<T>*)bin.dens4);
    }
    launch_fill_u32(&bin.cnt->n_fix, 2, 0u, s);
    hipLaunchKernelGGL(k_redo_list, dim3(wave_grid(bin.tile_cap, 4)), dim3(256), 0, s,
                       (const Tile*)bin.tiles, (const unsigned long long*)bin.ntiles,
                       (const uint32_t*)bin.boxph, nb, bin.fredo, bin.cnt, bin.tmpidx);
    launch_hmax_pyramid<T>(bin, sc, s);
    BinPtrs bf = bin;
    bf.tflag = bin.fredo;
    launch_tasks<T>(bf, sc, 2, true, s);
    KArgs<T> ar = make_args<T>(bin, sc);
    ar.out = (T*)bin.f_out;
    ar.gout = (T*)bin.g_out;
    ar.iout = bin.f_int;
    ar.order = bin.tmpidx;
    ar.ntask = &bin.cnt->n_fix;
    ar.xcd_split = 0;
    return launch_loop<L_FORCE, T>(ar, MODE_QUEUE, lds_cap, 2, s);
}
template int launch_single<float>(const BinPtrs&, const Scheme&, int, int, hipStream_t);
template int launch_single<double>(const BinPtrs&, const Scheme&, int, int, hipStream_t);

// ------------------------------------------------ time-dependent switches

// Viscosity switch after the density loop (Sec. 2.1.3, Eq. 12-16), per
// binned particle s (p = perm[s] its caller index): S = H^2 max(0, -(div v -
// div v_prev) / dt), alpha_loc = alpha_max S / (v_sig_prev^2 + S); alpha_V
// jumps up to alpha_loc or relaxes towards it as exp(-l c dt / H), floored
// at alpha_min; B = |div v| / (|div v| + |curl v| + bal_eps c / H).
// aux4[s] = (alpha_V(t + dt), B, 0, 0).
template <typename T>
__global__ void k_switch_visc(int64_t n, const int32_t* __restrict__ perm,
                              const T* __restrict__ div_v, const T* __restrict__ div_prev,
                              const T* __restrict__ cx, const T* __restrict__ cy,
                              const T* __restrict__ cz, const T* __restrict__ vsig_prev,
                              const T* __restrict__ av_in, const T* __restrict__ hs,
                              const V4<T>* __restrict__ vel4, SwitchConsts sw, T eps, T gamma,
                              V4<T>* __restrict__ aux4) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t p = perm[s];
    const T H = eps * hs[s];
    const T c = sqrt(gamma * (gamma - (T)1) * vel4[s].w);
    const T dt = (T)sw.dt;
    const T ddiv = (div_v[p] - div_prev[p]) / dt;
    const T S = H * H * (ddiv < (T)0 ? -ddiv : (T)0);
    const T vs = vsig_prev[p];
    const T aloc = S > (T)0 ? (T)sw.av_max * S / (vs * vs + S) : (T)0;
    T al = av_in[p];
    al = aloc >= al ? aloc : aloc + (al - aloc) * exp(-(T)sw.ell * c * dt / H);
    if (al < (T)sw.av_min) al = (T)sw.av_min;
    const T dd = fabs(div_v[p]);
    const T w = sqrt(cx[p] * cx[p] + cy[p] * cy[p] + cz[p] * cz[p]);
    const T den = dd + w + (T)sw.bal_eps * c / H;
    aux4[s] = V4<T>{al, den > (T)0 ? dd / den : (T)0, (T)0, (T)0};
}

// Conduction switch after the gradient loop (Sec. 2.1.4, Eq. 21, 23-24):
// one explicit step d alpha_c/dt = beta_c H lap u / sqrt(u) - (alpha_c -
// alpha_c,min) v_sig / H, then clamped to [alpha_c,min, alpha_c,max (1 -
// alpha_V,ngb / alpha_V,max)].  gsw: the gradient outputs (v_sig, lap u,
// alpha_V,ngb), binned.  Writes aux4[s].z.
template <typename T>
__global__ void k_switch_cond(int64_t n, const int32_t* __restrict__ perm,
                              const T* __restrict__ ac_in, const T* __restrict__ hs,
                              const V4<T>* __restrict__ vel4, const T* __restrict__ gsw,
                              SwitchConsts sw, T eps, V4<T>* __restrict__ aux4) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t p = perm[s];
    const T H = eps * hs[s];
    const T u = vel4[s].w;
    const T vs = gsw[s], lap = gsw[n + s], avn = gsw[2 * n + s];
    const T a0 = ac_in[p];
    const T src = u > (T)0 ? (T)sw.beta_c * H * lap / sqrt(u) : (T)0;
    const T rate = src - (a0 - (T)sw.ac_min) * vs / H;
    T a = a0 + (T)sw.dt * rate;
    const T amax = (T)sw.ac_max * ((T)1 - avn / (T)sw.av_max);
    if (a > amax) a = amax;
    if (a < (T)sw.ac_min) a = (T)sw.ac_min;
    aux4[s].z = a;
}

// The switch values back to the caller's order (p: caller index, rank[p]
// its binned position); balsara and av_ngb may be null.
template <typename T>
__global__ void k_switch_out(int64_t n, const int32_t* __restrict__ rank,
                             const V4<T>* __restrict__ aux4, const T* __restrict__ gsw,
                             T* __restrict__ av, T* __restrict__ ac, T* __restrict__ balsara,
                             T* __restrict__ av_ngb) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t s = rank[p];
    const V4<T> x = aux4[s];
    av[p] = x.x;
    ac[p] = x.z;
    if (balsara) balsara[p] = x.y;
    if (av_ngb) av_ngb[p] = gsw[2 * n + s];
}

// The gradient and force loops with switches over the force task lists
// (built first by launch_gf_tasks): viscosity switch, gradient loop,
// conduction switch, force loop.  aux4 (the adjoint scratch region, free
// outside the backward pass) holds (alpha_V, B, alpha_c, 0) per particle;
// g_out receives v_sig, lap u and alpha_V,ngb.
template <typename T>
int launch_switch_loops(const BinPtrs& b, const Scheme& sc, const SwitchConsts& sw,
                        const swsph_density_out* d, const swsph_switch_state* st, int mode,
                        int lds_cap, hipStream_t s) {
    if (b.n <= 0) return 0;
    const unsigned blocks = (unsigned)((b.n + 255) / 256);
    V4<T>* aux4 = (V4<T>*)b.adj;
    hipLaunchKernelGGL(k_switch_visc<T>, dim3(blocks), dim3(256), 0, s, b.n, b.perm,
                       (const T*)d->div_v, (const T*)st->div_v_prev, (const T*)d->curl_x,
                       (const T*)d->curl_y, (const T*)d->curl_z, (const T*)st->v_sig_prev,
                       (const T*)st->alpha_v, (const T*)b.hs, (const V4<T>*)b.vel4, sw,
                       (T)sc.eps, (T)sc.gamma, aux4);
    KArgs<T> a = make_args<T>(b, sc);
    a.aux4 = aux4;
    a.gout = (T*)b.g_out;
    timer_begin(sc.timer, 1, s);
    int r = launch_loop<L_GSW, T>(a, mode, lds_cap, 1, s);
    timer_end(sc.timer, 1, s);
    if (r) return r;
    hipLaunchKernelGGL(k_switch_cond<T>, dim3(blocks), dim3(256), 0, s, b.n, b.perm,
                       (const T*)st->alpha_c, (const T*)b.hs, (const V4<T>*)b.vel4,
                       (const T*)b.g_out, sw, (T)sc.eps, aux4);
    a.out = (T*)b.f_out;
    a.iout = b.f_int;
    timer_begin(sc.timer, 2, s);
    r = launch_loop<L_FSW, T>(a, mode, lds_cap, 2, s);
    timer_end(sc.timer, 2, s);
    if (r) return r;
    hipLaunchKernelGGL(k_switch_out<T>, dim3(blocks), dim3(256), 0, s, b.n, b.rank,
                       (const V4<T>*)aux4, (const T*)b.g_out, (T*)st->alpha_v, (T*)st->alpha_c,
                       (T*)st->balsara, (T*)st->alpha_v_ngb);
    return 0;
}
template int launch_switch_loops<float>(const BinPtrs&, const Scheme&, const SwitchConsts&,
                                        const swsph_density_out*, const swsph_switch_state*, int,
                                        int, hipStream_t);
template int launch_switch_loops<double>(const BinPtrs&, const Scheme&, const SwitchConsts&,
                                         const swsph_density_out*, const swsph_switch_state*,
                                         int, int, hipStream_t);

// ------------------------------------------------- per-particle preparation

// Gather the caller's density results (original order) into binned order:
// hs = h, dens4 = (rho, f, c, A) with c = sqrt(gamma (gamma-1) u) and
// A = f P / rho^2 = f (gamma-1) u / rho.
template <typename T>
__global__ void k_prep_dens(int64_t n, const int32_t* __restrict__ perm, const T* __restrict__ h,
                            const T* __restrict__ rho, const T* __restrict__ f,
                            const V4<T>* __restrict__ vel4, T gamma, T* __restrict__ hs,
                            V4<T>* __restrict__ dens4) {
    int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int32_t p = perm[s];
    const T u = vel4[s].w;
    const T r = rho[p], ff = f[p];
    hs[s] = h[p];
    const T gm1 = gamma - (T)1;
    dens4[s] = V4<T>{r, ff, sqrt(gamma * gm1 * u), ff * gm1 * u / r};
}

template <typename T>
void launch_prep_dens(const BinPtrs& b, const Scheme& sc, const swsph_density_out* d,
                      hipStream_t s) {
    if (b.n <= 0) return;
    hipLaunchKernelGGL(k_prep_dens<T>, dim3((unsigned)((b.n + 255) / 256)), dim3(256), 0, s, b.n,
                       b.perm, (const T*)d->h, (const T*)d->rho, (const T*)d->f,
                       (const V4<T>*)b.vel4, (T)sc.gamma, (T*)b.hs, (V4<T>*)b.dens4);
}
template void launch_prep_dens<float>(const BinPtrs&, const Scheme&, const swsph_density_out*,
                                      hipStream_t);
template void launch_prep_dens<double>(const BinPtrs&, const Scheme&, const swsph_density_out*,
                                       hipStream_t);

// Pyramid of per-cell maxima of the support radius H = eps h, levels 0..k
// of every box, in two passes.  The fine levels (HMAX_TOP + 1 .. k, and
// always level k) come from the particles: they are in Morton order, so the
// particles of a cell at any level are consecutive, and per level a
// wavefront takes the maximum over each run of lanes in the same cell
// (segmented scan with lane shuffles); only the last lane of a run raises
// the cell (atomic max, skipped when the cell already holds as much).  The
// coarse levels (at most 8^HMAX_TOP cells each) are then reduced from their
// children, one workgroup per box, level by level: the fine pass thus never
// has the whole grid contend for the few coarse cells.
constexpr int HMAX_TOP = 4;

__device__ __forceinline__ int hmax_fine_lo(int k) { return k < HMAX_TOP + 1 ? k : HMAX_TOP + 1; }
template <typename T>
__global__ void k_hmax(int64_t n, const int32_t* __restrict__ perm,
                       const uint32_t* __restrict__ keys, int32_t n_box,
                       const BoxInfo* __restrict__ boxtab, const T* __restrict__ hs, T eps,
                       float* __restrict__ pyr) {
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool have = s < n;
    const int lane = lane_id();
    int b = 0;
    uint32_t mort = 0;
    float H = 0.f;
    if (have) {
        const uint32_t key = keys[perm[s]];
        b = box_of_key(key, n_box, boxtab);
        mort = key - (uint32_t)boxtab[b].fine_off;
        H = (float)(eps * hs[s]) * (1.0f + 1e-6f);
    }
    const BoxInfo bi = boxtab[b];
    const int k = bi.k < 10 ? bi.k : 10;
    // all lanes run every fine level of the deepest box in the wavefront
    const int kmax = wave_max(have ? k - hmax_fine_lo(k) : 0);
    for (int up = 0; up <= kmax; ++up) {
        const int l = k - up;
        // cell id at this level; lanes past their box's root or without a
        // particle get ids no other lane has
        const bool mine = have && l >= hmax_fine_lo(k);
        const uint64_t cell = mine
            ? ((uint64_t)b << 32) | (uint64_t)(mort >> (3 * (k - l)))
            : ~(uint64_t)lane;
        float v = H;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            const float w = __shfl_up(v, o, WAVE);
            const uint64_t c = __shfl_up(cell, o, WAVE);
            if (lane >= o && c == cell) v = fmaxf(v, w);
        }
        const uint64_t next = __shfl_down(cell, 1, WAVE);
        const bool tail = lane == WAVE - 1 || next != cell;
        if (mine && tail) {
            float* c = &pyr[bi.pyr_off + pyr_level_off(l) + (mort >> (3 * (k - l)))];
            if (*c < v) atomicMax((int*)c, __float_as_int(v));
        }
    }
}

// The coarse levels hmax_fine_lo(k) - 1 .. 0 of each box from their
// children (cell c of level l has children 8c .. 8c + 7 at level l + 1).
__global__ void __launch_bounds__(256) k_hmax_coarse(int32_t n_box,
                                                     const BoxInfo* __restrict__ boxtab,
                                                     float* __restrict__ pyr) {
    for (int b = blockIdx.x; b < n_box; b += gridDim.x) {
        const BoxInfo bi = boxtab[b];
        const int k = bi.k < 10 ? bi.k : 10;
        for (int l = hmax_fine_lo(k) - 1; l >= 0; --l) {
            float* lv = pyr + bi.pyr_off + pyr_level_off(l);
            const float* ch = pyr + bi.pyr_off + pyr_level_off(l + 1);
            const int64_t nc = int64_t(1) << (3 * l);
            for (int64_t c = threadIdx.x; c < nc; c += blockDim.x) {
                float v = 0.f;
#pragma unroll
                for (int j = 0; j < 8; ++j) v = fmaxf(v, ch[8 * c + j]);
                lv[c] = v;
            }
            __syncthreads();  // level l complete before level l - 1 reads it
        }
    }
}

template <typename T>
void launch_hmax_pyramid(const BinPtrs& b, const Scheme& sc, hipStream_t s) {
    launch_fill_u32(b.hmaxpyr, b.n_pyr, 0u, s);
    if (b.n <= 0) return;
    hipLaunchKernelGGL(k_hmax<T>, dim3((unsigned)((b.n + 255) / 256)), dim3(256), 0, s, b.n,
                       b.perm, b.keys, b.n_box, b.boxtab, (const T*)b.hs, (T)sc.eps, b.hmaxpyr);
    const unsigned g = (unsigned)std::min<int64_t>(b.n_box, 4096);
    hipLaunchKernelGGL(k_hmax_coarse, dim3(g > 0 ? g : 1), dim3(256), 0, s, b.n_box, b.boxtab,
                       b.hmaxpyr);
}
template void launch_hmax_pyramid<float>(const BinPtrs&, const Scheme&, hipStream_t);
template void launch_hmax_pyramid<double>(const BinPtrs&, const Scheme&, hipStream_t);

}  // namespace swsph
