/*
 * swsph_oracle.c -- FP64 CPU reference for the SPH neighbour loops.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP library (no headers, helpers, tables or constants): every
 * formula below is written out again from the paper's equations.
 *
 * What it computes (paper: "Task-parallelism in SWIFT for heterogeneous
 * compute architectures", Section 2.1):
 *
 *   kernel      M4 cubic spline on support H = eps*h (Sec. 2.1.1; eps = 2 in
 *               all the paper's tests, Sec. 3.1):
 *                 W(r,h) = (8/pi) H^-3 w(r/H),
 *                 w(q) = 1 - 6q^2 + 6q^3 (q < 1/2), 2(1-q)^3 (1/2 <= q < 1)
 *   density     n_i = sum_j W(r_ij,h_i) (Eq. 5), dn_i/dh (Eq. 6, with the
 *               scalar radial derivative), rho_i = sum_j m_j W_ij (Eq. 2),
 *               drho_i/dh; h_i solves h^3 n_i(h) = eta^3 (the number-density
 *               target of Sec. 2.1.2) by safeguarded Newton iteration;
 *               div v and curl v (Eq. 3-4, difference form);
 *               f_i = 1 / (1 + h_i/(3 rho_i) drho_i/dh) (Eq. 8, grad-h factor
 *               applied as a divisor);
 *               neighbour count = #{j != i : r_ij^2 < H_i^2} evaluated in
 *               binary32 (see nngb_pred below).
 *   gradient    v_sig,i = max(2 c_i, max_j (c_i + c_j - beta mu_ij))
 *               (Eq. 10-11) and the Laplacian of u
 *               2 sum_j (m_j/rho_j)(u_i-u_j) (1/r) dW/dr(r,h_i), the inputs of
 *               the dissipation switches (Eq. 13, Eq. 21), Sec. 2.1.3.
 *   force       Eq. 17-18 with the grad-h factors, plus the pairwise
 *               viscosity of Eq. 7 and Eq. 9-11 (alpha constant, B = 1):
 *                 a_i  = -sum_j m_j [A_i G_i + A_j G_j + nu/2 (f_i G_i + f_j G_j)]
 *                 du_i =  sum_j m_j [A_i v_ij.G_i + nu/4 v_ij.(f_i G_i + f_j G_j)]
 *               A = f P / rho^2, P = (gamma-1) rho u, c = sqrt(gamma(gamma-1)u),
 *               G_k = grad_i W(r_ij, h_k), mu = min(0, v_ij . r_hat),
 *               v_sig = c_i + c_j - beta mu, nu = -alpha mu v_sig/(rho_i+rho_j).
 *               Pairs: j != i with r < max(H_i, H_j).
 *   switches    the time-dependent dissipation switches of Sec. 2.1.3-2.1.4
 *               (Eq. 12-16 viscosity coefficient and Balsara factor, Eq. 19-24
 *               artificial conduction): per-particle updates and the force
 *               loop with alpha_ij and conduction (orc_switch_visc,
 *               orc_alpha_ngb, orc_switch_cond, orc_force_sw; readings of
 *               the garbled equations stated there).
 *
 * Conventions: r_ij = x_i - x_j - s (minimum periodic image s), v_ij = v_i - v_j.
 * The self term j = i enters n, rho and their h-derivatives, and nothing
 * else.  Inputs are float64 arrays (the callers widen float32 data exactly).
 *
 * Neighbour search has two modes that must give the same sets:
 *   brute   every pair, the definition;
 *   cells   a uniform grid of the periodic box, all cells within reach;
 *           a cell is skipped only when its minimum-image distance to x_i
 *           already exceeds the search radius.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_VERSION 1
#define ORC_PI 3.14159265358979323846

typedef struct {
    double eta;      /* resolution: h^3 n(h) = eta^3 */
    double eps;      /* support radius H = eps * h */
    double gamma;    /* adiabatic index */
    double alpha;    /* viscosity coefficient */
    double beta;     /* signal-velocity coefficient */
    double tol;      /* Newton stop: |G - eta^3| <= tol * eta^3 */
    int32_t max_iter;
    int32_t visc;    /* 0: viscosity off */
    int32_t mode;    /* 0: brute force, 1: cell grid */
    int32_t ncell;   /* cells per dimension in cell mode (0: choose) */
} orc_params;

/* ---------------------------------------------------------------- kernel */

static double w_q(double q) {
    if (q < 0.5) return 1.0 - 6.0 * q * q + 6.0 * q * q * q;
    if (q < 1.0) { double t = 1.0 - q; return 2.0 * t * t * t; }
    return 0.0;
}
static double dw_q(double q) {
    if (q < 0.5) return -12.0 * q + 18.0 * q * q;
    if (q < 1.0) { double t = 1.0 - q; return -6.0 * t * t; }
    return 0.0;
}
static double d2w_q(double q) {
    if (q < 0.5) return -12.0 + 36.0 * q;
    if (q < 1.0) return 12.0 * (1.0 - q);
    return 0.0;
}

/* W(r,h), dW/dr, dW/dh for support H = eps h. */
static double kW(double r, double h, double eps) {
    double H = eps * h;
    return (8.0 / ORC_PI) / (H * H * H) * w_q(r / H);
}
static double kdWdr(double r, double h, double eps) {
    double H = eps * h;
    return (8.0 / ORC_PI) / (H * H * H * H) * dw_q(r / H);
}
static double kdWdh(double r, double h, double eps) {
    return -(3.0 * kW(r, h, eps) + r * kdWdr(r, h, eps)) / h;
}

int orc_version(void) { return ORC_VERSION; }

/* which: 0 w, 1 w', 2 w'', 3 W(r,h), 4 dW/dr, 5 dW/dh  (a = q or r, b = h) */
void orc_kernel_eval(int which, int64_t n, const double* a, double b, double eps,
                     double* out) {
    for (int64_t k = 0; k < n; ++k) {
        switch (which) {
            case 0: out[k] = w_q(a[k]); break;
            case 1: out[k] = dw_q(a[k]); break;
            case 2: out[k] = d2w_q(a[k]); break;
            case 3: out[k] = kW(a[k], b, eps); break;
            case 4: out[k] = kdWdr(a[k], b, eps); break;
            default: out[k] = kdWdh(a[k], b, eps); break;
        }
    }
}

/* ------------------------------------------------------- neighbour search */

typedef struct {
    int64_t n;
    const double *x, *y, *z;
    double L;
    int mode;
    int nc;
    double w;
    int64_t* cstart;  /* nc^3 + 1 */
    int64_t* citem;   /* n */
} orc_grid;

typedef struct {
    int64_t j;
    double dx, dy, dz, r;
    double sx, sy, sz; /* periodic image added to x_j */
} orc_nb;

typedef struct {
    orc_nb* a;
    int64_t n, cap;
} orc_list;

static void list_push(orc_list* l, orc_nb v) {
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 256;
        l->a = (orc_nb*)realloc(l->a, (size_t)l->cap * sizeof(orc_nb));
    }
    l->a[l->n++] = v;
}

static int cell_of(double x, double w, int nc) {
    int c = (int)floor(x / w);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

static int grid_build(orc_grid* g, int64_t n, const double* x, const double* y,
                      const double* z, double L, int mode, int nc) {
    memset(g, 0, sizeof(*g));
    g->n = n; g->x = x; g->y = y; g->z = z; g->L = L; g->mode = mode;
    if (mode == 0) return 0;
    if (nc <= 0) {
        /* about 8 particles per cell */
        nc = (int)floor(cbrt((double)n / 8.0));
        if (nc < 1) nc = 1;
        if (nc > 256) nc = 256;
    }
    g->nc = nc;
    g->w = L / nc;
    int64_t ncells = (int64_t)nc * nc * nc;
    g->cstart = (int64_t*)calloc((size_t)ncells + 1, sizeof(int64_t));
    g->citem = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t* key = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!g->cstart || !g->citem || !key) return -1;
    for (int64_t i = 0; i < n; ++i) {
        int cx = cell_of(x[i], g->w, nc), cy = cell_of(y[i], g->w, nc),
            cz = cell_of(z[i], g->w, nc);
        key[i] = ((int64_t)cz * nc + cy) * nc + cx;
        g->cstart[key[i] + 1]++;
    }
    for (int64_t c = 0; c < ncells; ++c) g->cstart[c + 1] += g->cstart[c];
    int64_t* fill = (int64_t*)malloc((size_t)ncells * sizeof(int64_t));
    memcpy(fill, g->cstart, (size_t)ncells * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) g->citem[fill[key[i]]++] = i;
    free(fill);
    free(key);
    return 0;
}

static void grid_free(orc_grid* g) {
    free(g->cstart);
    free(g->citem);
}

/* Minimum-image displacement x_i - x_j - s along one axis. */
static double min_image(double xi, double xj, double L, double* s) {
    double d = xi - xj;
    *s = 0.0;
    if (d > 0.5 * L) { *s = L; d -= L; }
    else if (d < -0.5 * L) { *s = -L; d += L; }
    return d;
}

static int consider(const orc_grid* g, int64_t i, int64_t j, double R,
                    const double* Hj, orc_list* out) {
    orc_nb v;
    v.j = j;
    v.dx = min_image(g->x[i], g->x[j], g->L, &v.sx);
    v.dy = min_image(g->y[i], g->y[j], g->L, &v.sy);
    v.dz = min_image(g->z[i], g->z[j], g->L, &v.sz);
    v.r = sqrt(v.dx * v.dx + v.dy * v.dy + v.dz * v.dz);
    double lim = R;
    if (Hj && Hj[j] > lim) lim = Hj[j];
    if (v.r < lim) { list_push(out, v); return 1; }
    return 0;
}

/* Minimum-image distance from point p to the cell interval [c*w, (c+1)*w). */
static double axis_gap(double p, int c, double w, double L) {
    double lo = c * w, hi = (c + 1) * w;
    double best = 1e300;
    for (int k = -1; k <= 1; ++k) {
        double a = lo + k * L, b = hi + k * L, d;
        if (p < a) d = a - p; else if (p > b) d = p - b; else d = 0.0;
        if (d < best) best = d;
    }
    return best;
}

/*
 * All j (including i itself) with r_ij < max(R, Hj[j]) (Hj may be NULL), and
 * Hmax >= every Hj[j] (only used to size the cell reach).
 */
static void gather(const orc_grid* g, int64_t i, double R, const double* Hj,
                   double Hmax, orc_list* out) {
    out->n = 0;
    if (g->mode == 0) {
        for (int64_t j = 0; j < g->n; ++j) consider(g, i, j, R, Hj, out);
        return;
    }
    double Rs = R;
    if (Hj && Hmax > Rs) Rs = Hmax;
    int nc = g->nc;
    int reach = (int)ceil(Rs / g->w);
    int ci[3] = {cell_of(g->x[i], g->w, nc), cell_of(g->y[i], g->w, nc),
                 cell_of(g->z[i], g->w, nc)};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        if (2 * reach + 1 >= nc) { lo[d] = 0; hi[d] = nc - 1; }
        else { lo[d] = ci[d] - reach; hi[d] = ci[d] + reach; }
    }
    for (int a = lo[2]; a <= hi[2]; ++a) {
        int cz = ((a % nc) + nc) % nc;
        double gz = axis_gap(g->z[i], cz, g->w, g->L);
        for (int b = lo[1]; b <= hi[1]; ++b) {
            int cy = ((b % nc) + nc) % nc;
            double gy = axis_gap(g->y[i], cy, g->w, g->L);
            for (int c = lo[0]; c <= hi[0]; ++c) {
                int cx = ((c % nc) + nc) % nc;
                double gx = axis_gap(g->x[i], cx, g->w, g->L);
                if (sqrt(gx * gx + gy * gy + gz * gz) >= Rs) continue;
                int64_t cell = ((int64_t)cz * nc + cy) * nc + cx;
                for (int64_t k = g->cstart[cell]; k < g->cstart[cell + 1]; ++k)
                    consider(g, i, g->citem[k], R, Hj, out);
            }
        }
    }
}

/*
 * Neighbour predicate in binary32 (used for the integer neighbour counts, so
 * that an FP32 implementation can reproduce them bit for bit):
 *   xs = fl32(x_j + s), dx = fl32(x_i - xs) (same for y, z),
 *   r2 = fl32(fl32(fl32(dx*dx) + fl32(dy*dy)) + fl32(dz*dz)),
 *   H  = fl32(eps * h), H2 = fl32(H*H),  neighbour iff r2 < H2.
 * Compiled with -ffp-contract=off so no product is fused into an addition.
 */
static float r2_f32(const orc_grid* g, int64_t i, const orc_nb* v) {
    float xi = (float)g->x[i], yi = (float)g->y[i], zi = (float)g->z[i];
    float xs = (float)g->x[v->j] + (float)v->sx;
    float ys = (float)g->y[v->j] + (float)v->sy;
    float zs = (float)g->z[v->j] + (float)v->sz;
    float dx = xi - xs, dy = yi - ys, dz = zi - zs;
    float a = dx * dx, b = dy * dy, c = dz * dz;
    float s = a + b;
    return s + c;
}
static float H2_f32(float h, float eps) {
    float H = eps * h;
    return H * H;
}

/* ------------------------------------------------------------ density */

/* n(h) and dn/dh over the list (entries with r < eps h). */
static void nsum(const orc_list* l, double h, double eps, double* n, double* dn) {
    double H = eps * h, a = 0.0, b = 0.0;
    for (int64_t k = 0; k < l->n; ++k) {
        double r = l->a[k].r;
        if (r < H) {
            a += kW(r, h, eps);
            b += kdWdh(r, h, eps);
        }
    }
    *n = a;
    *dn = b;
}

/*
 * Solve G(h) = h^3 n(h) = eta^3 for particle i (Sec. 2.1.2).  G is
 * non-decreasing in h, G(0+) = 8/(pi eps^3) < eta^3 for the parameters in
 * use, so the root is unique.  Safeguarded Newton: a bracket [lo, hi] with
 * G(lo) < eta^3 <= G(hi); a Newton step leaving the bracket is replaced by
 * bisection.  Returns the iteration count, or -1 when H would reach L/2.
 */
static int solve_h(const orc_grid* g, int64_t i, double hguess, const orc_params* p,
                   orc_list* l, double* hout, int* conv) {
    const double T = p->eta * p->eta * p->eta;
    double R = p->eps * hguess * 1.25;
    if (!(R > 0)) R = 0.1 * g->L;
    for (;;) {
        if (R >= 0.5 * g->L) R = 0.5 * g->L * (1.0 - 1e-12);
        gather(g, i, R, NULL, 0.0, l);
        double hi = R / p->eps, n, dn;
        nsum(l, hi, p->eps, &n, &dn);
        if (hi * hi * hi * n >= T) break;
        if (R >= 0.5 * g->L * (1.0 - 1e-9)) return -1;
        R *= 1.6;
    }
    double lo = 0.0, hi = R / p->eps;
    double h = hguess;
    if (!(h > lo && h < hi)) h = 0.5 * (lo + hi);
    *conv = 0;
    int it;
    for (it = 1; it <= p->max_iter; ++it) {
        double n, dn;
        nsum(l, h, p->eps, &n, &dn);
        double G = h * h * h * n;
        double dG = 3.0 * h * h * n + h * h * h * dn;
        if (fabs(G - T) <= p->tol * T) { *conv = 1; break; }
        if (G < T) lo = h; else hi = h;
        double hn = h - (G - T) / dG;
        if (!(dG > 0) || !(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
        if (hi - lo <= 4.0 * DBL_EPSILON * hi) { *conv = 1; break; }
        h = hn;
    }
    *hout = h;
    return it;
}

typedef struct {
    double *h, *rho, *rho_dh, *wcount, *wcount_dh, *div_v, *curl_x, *curl_y,
        *curl_z, *f;
    int32_t *nngb, *iters;
} orc_density_out;

static void density_at(const orc_grid* g, int64_t i, double h, const double* vx,
                       const double* vy, const double* vz, const double* m,
                       const orc_params* p, const orc_list* l,
                       const orc_density_out* o) {
    double eps = p->eps, H = eps * h;
    double n = 0, dn = 0, rho = 0, drho = 0, dv = 0, cx = 0, cy = 0, cz = 0;
    int32_t cnt = 0;
    float H2 = H2_f32((float)h, (float)eps);
    for (int64_t k = 0; k < l->n; ++k) {
        const orc_nb* v = &l->a[k];
        int64_t j = v->j;
        if (j != i && r2_f32(g, i, v) < H2) cnt++;
        if (!(v->r < H)) continue;
        double W = kW(v->r, h, eps), Wh = kdWdh(v->r, h, eps);
        n += W;
        dn += Wh;
        rho += m[j] * W;
        drho += m[j] * Wh;
        if (j == i || v->r == 0.0) continue;
        /* grad_i W_ij = r_hat dW/dr */
        double gr = kdWdr(v->r, h, eps) / v->r;
        double gx = v->dx * gr, gy = v->dy * gr, gz = v->dz * gr;
        double ux = vx[i] - vx[j], uy = vy[i] - vy[j], uz = vz[i] - vz[j];
        dv += m[j] * (ux * gx + uy * gy + uz * gz);
        cx += m[j] * (uy * gz - uz * gy);
        cy += m[j] * (uz * gx - ux * gz);
        cz += m[j] * (ux * gy - uy * gx);
    }
    if (o->h) o->h[i] = h;
    if (o->rho) o->rho[i] = rho;
    if (o->rho_dh) o->rho_dh[i] = drho;
    if (o->wcount) o->wcount[i] = n;
    if (o->wcount_dh) o->wcount_dh[i] = dn;
    /* div v = -(1/rho) sum m_j v_ij . grad_i W ; curl v = (1/rho) sum m_j v_ij x grad_i W */
    if (o->div_v) o->div_v[i] = -dv / rho;
    if (o->curl_x) o->curl_x[i] = cx / rho;
    if (o->curl_y) o->curl_y[i] = cy / rho;
    if (o->curl_z) o->curl_z[i] = cz / rho;
    if (o->f) o->f[i] = 1.0 / (1.0 + h * drho / (3.0 * rho));
    if (o->nngb) o->nngb[i] = cnt;
}

/*
 * Density loop for the particles listed in idx (all when idx == NULL).
 * h_fixed != NULL: use those smoothing lengths (no Newton), else solve.
 * h_guess may be NULL (the guess then comes from the local cell occupancy).
 * Returns the number of particles that failed (reach or no convergence).
 */
int64_t orc_density(int64_t n, const double* x, const double* y, const double* z,
                    const double* vx, const double* vy, const double* vz,
                    const double* m, double L, const orc_params* p,
                    const double* h_fixed, const double* h_guess, int64_t nidx,
                    const int64_t* idx, double* h, double* rho, double* rho_dh,
                    double* wcount, double* wcount_dh, double* div_v,
                    double* curl_x, double* curl_y, double* curl_z, double* f,
                    int32_t* nngb, int32_t* iters) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, p->mode, p->ncell)) return -1;
    orc_density_out o = {h, rho, rho_dh, wcount, wcount_dh, div_v, curl_x,
                         curl_y, curl_z, f, nngb, iters};
    int64_t cnt = (idx ? nidx : n), bad = 0;
    double hdef = p->eta * L / cbrt((double)(n > 0 ? n : 1));
    /* default guess: eta times the mean spacing in the particle's own cell */
    double* hcell = NULL;
    if (g.mode == 1) {
        int64_t nc3 = (int64_t)g.nc * g.nc * g.nc;
        hcell = (double*)malloc((size_t)nc3 * sizeof(double));
        for (int64_t c = 0; c < nc3; ++c) {
            int64_t k = g.cstart[c + 1] - g.cstart[c];
            hcell[c] = k > 0 ? p->eta * g.w / cbrt((double)k) : hdef;
        }
    }
#pragma omp parallel reduction(+ : bad)
    {
        orc_list l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < cnt; ++k) {
            int64_t i = idx ? idx[k] : k;
            double hi;
            int it = 0, conv = 1;
            if (h_fixed) {
                hi = h_fixed[i];
                double R = p->eps * hi;
                gather(&g, i, R, NULL, 0.0, &l);
            } else {
                double hg = hdef;
                if (h_guess && h_guess[i] > 0) hg = h_guess[i];
                else if (hcell) {
                    int nc = g.nc;
                    int64_t c = ((int64_t)cell_of(z[i], g.w, nc) * nc +
                                 cell_of(y[i], g.w, nc)) * nc + cell_of(x[i], g.w, nc);
                    hg = hcell[c];
                }
                it = solve_h(&g, i, hg, p, &l, &hi, &conv);
                if (it < 0) { bad++; if (iters) iters[i] = -1; continue; }
                if (!conv) bad++;
            }
            density_at(&g, i, hi, vx, vy, vz, m, p, &l, &o);
            if (iters) iters[i] = conv ? it : -it;
        }
        free(l.a);
    }
    free(hcell);
    grid_free(&g);
    return bad;
}

/* ------------------------------------------------------------ gradient */

int64_t orc_gradient(int64_t n, const double* x, const double* y, const double* z,
                     const double* vx, const double* vy, const double* vz,
                     const double* u, const double* m, double L,
                     const orc_params* p, const double* h, const double* rho,
                     int64_t nidx, const int64_t* idx, double* vsig, double* lapu) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, p->mode, p->ncell)) return -1;
    const double gg = p->gamma * (p->gamma - 1.0);
    int64_t cnt = (idx ? nidx : n);
#pragma omp parallel
    {
        orc_list l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < cnt; ++k) {
            int64_t i = idx ? idx[k] : k;
            double H = p->eps * h[i];
            gather(&g, i, H, NULL, 0.0, &l);
            double ci = sqrt(gg * u[i]);
            double vs = 2.0 * ci, lap = 0.0;
            for (int64_t q = 0; q < l.n; ++q) {
                const orc_nb* v = &l.a[q];
                int64_t j = v->j;
                if (j == i || v->r == 0.0) continue;
                double cj = sqrt(gg * u[j]);
                double vr = (vx[i] - vx[j]) * v->dx + (vy[i] - vy[j]) * v->dy +
                            (vz[i] - vz[j]) * v->dz;
                double mu = vr < 0.0 ? vr / v->r : 0.0;
                double s = ci + cj - p->beta * mu;
                if (s > vs) vs = s;
                lap += (m[j] / rho[j]) * (u[i] - u[j]) * kdWdr(v->r, h[i], p->eps) / v->r;
            }
            vsig[i] = vs;
            lapu[i] = 2.0 * lap;
        }
        free(l.a);
    }
    grid_free(&g);
    return 0;
}

/* --------------------------------------------------------------- force */

static double max_of(const double* a, int64_t n) {
    double v = 0.0;
    for (int64_t k = 0; k < n; ++k) if (a[k] > v) v = a[k];
    return v;
}

/*
 * Force loop for the particles listed in idx (all when idx == NULL).
 * h, rho, f: per-particle density results for all n particles.
 * nint (nullable) receives #{j != i : r < max(H_i, H_j)} (FP64 test).
 */
int64_t orc_force(int64_t n, const double* x, const double* y, const double* z,
                  const double* vx, const double* vy, const double* vz,
                  const double* u, const double* m, double L, const orc_params* p,
                  const double* h, const double* rho, const double* f,
                  int64_t nidx, const int64_t* idx, double* ax, double* ay,
                  double* az, double* dudt, int32_t* nint) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, p->mode, p->ncell)) return -1;
    const double gm1 = p->gamma - 1.0, gg = p->gamma * gm1;
    double* Hs = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t k = 0; k < n; ++k) Hs[k] = p->eps * h[k];
    double Hmax = max_of(Hs, n);
    int64_t cnt = (idx ? nidx : n);
#pragma omp parallel
    {
        orc_list l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < cnt; ++k) {
            int64_t i = idx ? idx[k] : k;
            gather(&g, i, Hs[i], Hs, Hmax, &l);
            double Ai = f[i] * gm1 * u[i] / rho[i];
            double ci = sqrt(gg * u[i]);
            double sx = 0, sy = 0, sz = 0, su = 0;
            int32_t c = 0;
            for (int64_t q = 0; q < l.n; ++q) {
                const orc_nb* v = &l.a[q];
                int64_t j = v->j;
                if (j == i) continue;
                c++;
                if (v->r == 0.0) continue;
                double Aj = f[j] * gm1 * u[j] / rho[j];
                double cj = sqrt(gg * u[j]);
                double ex = v->dx / v->r, ey = v->dy / v->r, ez = v->dz / v->r;
                /* scalar radial derivatives at each particle's own h; zero
                 * outside that particle's support */
                double gi = v->r < Hs[i] ? kdWdr(v->r, h[i], p->eps) : 0.0;
                double gj = v->r < Hs[j] ? kdWdr(v->r, h[j], p->eps) : 0.0;
                double wx = vx[i] - vx[j], wy = vy[i] - vy[j], wz = vz[i] - vz[j];
                double vdote = wx * ex + wy * ey + wz * ez;
                double nu = 0.0;
                if (p->visc) {
                    double mu = vdote < 0.0 ? vdote : 0.0;
                    double vsig = ci + cj - p->beta * mu;
                    nu = -p->alpha * mu * vsig / (rho[i] + rho[j]);
                }
                double fg = f[i] * gi + f[j] * gj;
                double sa = Ai * gi + Aj * gj + 0.5 * nu * fg;
                sx -= m[j] * sa * ex;
                sy -= m[j] * sa * ey;
                sz -= m[j] * sa * ez;
                su += m[j] * vdote * (Ai * gi + 0.25 * nu * fg);
            }
            ax[i] = sx; ay[i] = sy; az[i] = sz; dudt[i] = su;
            if (nint) nint[i] = c;
        }
        free(l.a);
    }
    free(Hs);
    grid_free(&g);
    return 0;
}

/* ------------------------------------------------ neighbour sets (tests) */

/*
 * For each listed particle i: the sorted indices j != i with
 * r_ij < max(R_i, (Hj ? Hj[j] : 0)) in FP64 (rad) -- used to check the cell
 * mode against brute force.  out_cnt[k] = count; out_list is row-major with
 * stride cap (entries beyond cap are dropped, count is still exact).
 */
static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}
int64_t orc_neighbour_sets(int64_t n, const double* x, const double* y,
                           const double* z, double L, int mode, int ncell,
                           const double* R, const double* Hj, int64_t nidx,
                           const int64_t* idx, int64_t cap, int64_t* out_cnt,
                           int64_t* out_list) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, mode, ncell)) return -1;
    double Hmax = Hj ? max_of(Hj, n) : 0.0;
#pragma omp parallel
    {
        orc_list l = {0, 0, 0};
        int64_t* tmp = NULL;
        int64_t tcap = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < nidx; ++k) {
            int64_t i = idx[k];
            gather(&g, i, R[i], Hj, Hmax, &l);
            if (l.n > tcap) { tcap = l.n; tmp = (int64_t*)realloc(tmp, (size_t)tcap * sizeof(int64_t)); }
            int64_t c = 0;
            for (int64_t q = 0; q < l.n; ++q) if (l.a[q].j != i) tmp[c++] = l.a[q].j;
            qsort(tmp, (size_t)c, sizeof(int64_t), cmp_i64);
            out_cnt[k] = c;
            for (int64_t q = 0; q < c && q < cap; ++q) out_list[k * cap + q] = tmp[q];
        }
        free(tmp);
        free(l.a);
    }
    grid_free(&g);
    return 0;
}

/*
 * Binary32 neighbour counts at given float32 smoothing lengths:
 * cnt[k] = #{j != i : r2_f32 < H2_f32(h_i)} for i = idx[k] (density/gradient
 * predicate) and, when cnt_sym != NULL, #{j != i : r2_f32 < max(H2_i, H2_j)}
 * (force predicate).
 */
int64_t orc_count_f32(int64_t n, const double* x, const double* y, const double* z,
                      double L, int mode, int ncell, double eps, const float* hf,
                      int64_t nidx, const int64_t* idx, int32_t* cnt,
                      int32_t* cnt_sym) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, mode, ncell)) return -1;
    double* Hs = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    /* search radius padded by a relative 1e-5 so the binary32 predicate
     * decides every pair near the edge */
    for (int64_t k = 0; k < n; ++k) Hs[k] = eps * (double)hf[k] * (1.0 + 1e-5);
    double Hmax = max_of(Hs, n);
#pragma omp parallel
    {
        orc_list l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < nidx; ++k) {
            int64_t i = idx[k];
            gather(&g, i, Hs[i], cnt_sym ? Hs : NULL, Hmax, &l);
            float H2i = H2_f32(hf[i], (float)eps);
            int32_t a = 0, b = 0;
            for (int64_t q = 0; q < l.n; ++q) {
                int64_t j = l.a[q].j;
                if (j == i) continue;
                float r2 = r2_f32(&g, i, &l.a[q]);
                if (r2 < H2i) a++;
                if (cnt_sym) {
                    float H2j = H2_f32(hf[j], (float)eps);
                    if (r2 < (H2i > H2j ? H2i : H2j)) b++;
                }
            }
            cnt[k] = a;
            if (cnt_sym) cnt_sym[k] = b;
        }
        free(l.a);
    }
    free(Hs);
    grid_free(&g);
    return 0;
}

/*
 * The same binary32 counts for every particle, with the force predicate
 * enumerated from both sides of each pair instead of by one search out to
 * the largest support in the box:
 *   cnt_sym_i = #{j != i : r2 < H2_i} + #{j != i : not (r2 < H2_i), r2 < H2_j},
 * the second term found by searching around each j within its own support.
 * r2 is always formed from i's side (x_i minus the image of x_j), exactly as
 * in orc_count_f32.  Costs one search per particle at its own radius, so it
 * stays cheap when the supports of a set span orders of magnitude.
 */
int64_t orc_count_f32_sym(int64_t n, const double* x, const double* y, const double* z,
                          double L, int mode, int ncell, double eps, const float* hf,
                          int32_t* cnt, int32_t* cnt_sym) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, mode, ncell)) return -1;
    double* Hs = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    int32_t* extra = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    for (int64_t k = 0; k < n; ++k) Hs[k] = eps * (double)hf[k] * (1.0 + 1e-5);
#pragma omp parallel
    {
        orc_list l = {0, 0, 0};
        /* pairs inside the support of i */
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            gather(&g, i, Hs[i], NULL, 0.0, &l);
            float H2i = H2_f32(hf[i], (float)eps);
            int32_t a = 0;
            for (int64_t q = 0; q < l.n; ++q) {
                if (l.a[q].j == i) continue;
                if (r2_f32(&g, i, &l.a[q]) < H2i) a++;
            }
            cnt[i] = a;
        }
        /* pairs inside the support of j only, credited to i */
#pragma omp for schedule(dynamic, 64)
        for (int64_t j = 0; j < n; ++j) {
            gather(&g, j, Hs[j], NULL, 0.0, &l);
            float H2j = H2_f32(hf[j], (float)eps);
            for (int64_t q = 0; q < l.n; ++q) {
                int64_t i = l.a[q].j;
                if (i == j) continue;
                /* the same pair seen from i: the image of x_j is shifted the
                 * opposite way */
                orc_nb w = l.a[q];
                w.j = j;
                w.sx = -w.sx; w.sy = -w.sy; w.sz = -w.sz;
                float r2 = r2_f32(&g, i, &w);
                float H2i = H2_f32(hf[i], (float)eps);
                if (!(r2 < H2i) && r2 < H2j) {
#pragma omp atomic
                    extra[i]++;
                }
            }
        }
        free(l.a);
    }
    if (cnt_sym)
        for (int64_t i = 0; i < n; ++i) cnt_sym[i] = cnt[i] + extra[i];
    free(extra);
    free(Hs);
    grid_free(&g);
    return 0;
}

/* ------------------------------------------------- local loss (FD checks) */

/*
 * L_S = sum_{i in S} w_i . a_i + c_i du_i/dt, where a and du/dt of the
 * particles in S are computed from scratch (Newton for every particle whose
 * density they use).  Used for central finite differences of the full
 * density -> force map: a perturbation of particle k only changes outputs
 * within two supports of k, so S can be that neighbourhood and the
 * difference L_S(+) - L_S(-) carries no cancellation from far particles.
 * Rbig must bound every support radius H_j of the particles involved.
 */
int64_t orc_loss_subset(int64_t n, const double* x, const double* y, const double* z,
                        const double* vx, const double* vy, const double* vz,
                        const double* u, const double* m, double L,
                        const orc_params* p, const double* h_guess, double Rbig,
                        int64_t ns, const int64_t* S, const double* wx,
                        const double* wy, const double* wz, const double* c,
                        double* loss) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, p->mode, p->ncell)) return -1;
    /* D = S and every particle within Rbig of S */
    char* inD = (char*)calloc((size_t)n, 1);
    orc_list l = {0, 0, 0};
    for (int64_t k = 0; k < ns; ++k) {
        gather(&g, S[k], Rbig, NULL, 0.0, &l);
        for (int64_t q = 0; q < l.n; ++q) inD[l.a[q].j] = 1;
    }
    free(l.a);
    int64_t nd = 0;
    for (int64_t k = 0; k < n; ++k) nd += inD[k];
    int64_t* D = (int64_t*)malloc((size_t)(nd > 0 ? nd : 1) * sizeof(int64_t));
    nd = 0;
    for (int64_t k = 0; k < n; ++k) if (inD[k]) D[nd++] = k;
    double* h = (double*)calloc((size_t)n, sizeof(double));
    double* rho = (double*)calloc((size_t)n, sizeof(double));
    double* f = (double*)calloc((size_t)n, sizeof(double));
    int64_t bad = orc_density(n, x, y, z, vx, vy, vz, m, L, p, NULL, h_guess, nd, D,
                              h, rho, NULL, NULL, NULL, NULL, NULL, NULL, NULL, f,
                              NULL, NULL);
    /* every particle a force of S reads must have been solved */
    double* ax = (double*)calloc((size_t)n, sizeof(double));
    double* ay = (double*)calloc((size_t)n, sizeof(double));
    double* az = (double*)calloc((size_t)n, sizeof(double));
    double* du = (double*)calloc((size_t)n, sizeof(double));
    /* outside D, h = 0: such particles then have an empty support, and they
     * are never within reach of S by the choice of Rbig */
    orc_force(n, x, y, z, vx, vy, vz, u, m, L, p, h, rho, f, ns, S, ax, ay, az, du,
              NULL);
    double acc = 0.0;
    for (int64_t k = 0; k < ns; ++k) {
        int64_t i = S[k];
        acc += wx[i] * ax[i] + wy[i] * ay[i] + wz[i] * az[i] + c[i] * du[i];
    }
    *loss = acc;
    free(inD); free(D); free(h); free(rho); free(f);
    free(ax); free(ay); free(az); free(du);
    grid_free(&g);
    return bad;
}

/* ------------------------------------ time-dependent dissipation switches */

/*
 * SPHENIX-type switches (Sec. 2.1.3, Eq. 12-16; Sec. 2.1.4, Eq. 19-24),
 * with these readings of the printed equations (several are garbled):
 *
 *   Eq. 13-15  S_i = H_i^2 max(0, -(div v_i(t+dt) - div v_i(t)) / dt),
 *              alpha_loc,i = alpha_V,max S_i / (v_sig,i^2 + S_i), v_sig,i the
 *              particle's signal speed of the previous gradient loop (the
 *              printed dt factor on alpha_loc is dropped: alpha_loc is a
 *              dimensionless target);
 *   Eq. 12     alpha_V relaxes towards alpha_loc on the time scale
 *              H_i / (l c_i): alpha(t+dt) = alpha_loc when alpha_loc >=
 *              alpha(t), else alpha_loc + (alpha(t) - alpha_loc)
 *              exp(-l c_i dt / H_i); then at least alpha_V,min;
 *   Eq. 16     B_i the Balsara factor |div v| / (|div v| + |curl v| +
 *              bal_eps c_i / H_i) (the paper names B without defining it);
 *   Eq. 24     alpha_c,max,i = alpha_c,max (1 - alpha_V,ngb,i / alpha_V,max),
 *              alpha_V,ngb,i the largest alpha_V over the particle's support
 *              (its own included);
 *   Eq. 21     d alpha_c,i / dt = beta_c H_i lap u_i / sqrt(u_i)
 *              - (alpha_c,i - alpha_c,min) v_sig,i / H_i (the printed extra
 *              alpha_c factor of the source term is dropped: with it
 *              alpha_c = 0 could never switch on; v_c,i read as the
 *              particle's signal speed); one explicit Euler step of dt,
 *              then clamped to [alpha_c,min, alpha_c,max,i] (Eq. 23);
 *   Eq. 20     alpha_c,ij = (P_i alpha_c,i + P_j alpha_c,j) / (P_i + P_j);
 *   Eq. 22     v_c,ij = |v_ij . r_hat| + sqrt(2 |P_i - P_j| / (rho_i + rho_j))
 *              (the relative velocity, so the pair term is symmetric);
 *   Eq. 19     du_i/dt += sum_j alpha_c,ij v_c,ij m_j (u_i - u_j)
 *              (f_i dW/dr(r,h_i) + f_j dW/dr(r,h_j)) / (rho_i + rho_j),
 *              the kernel gradients taken as scalar radial derivatives
 *              (negative: heat flows from the hotter particle);
 *   Eq. 16     alpha_ij = (alpha_V,i + alpha_V,j)/2 (B_i + B_j)/2 replaces
 *              the constant alpha in the viscosity of Eq. 9.
 */
typedef struct {
    double dt;       /* time step of the switch update */
    double av_max;   /* alpha_V,max (Eq. 13) */
    double av_min;   /* floor of alpha_V */
    double ell;      /* decay length l (Eq. 12; 0.05 in the paper) */
    double beta_c;   /* beta_c (Eq. 21) */
    double ac_min;   /* alpha_c,min (Eq. 21) */
    double ac_max;   /* alpha_c,max (Eq. 23-24) */
    double bal_eps;  /* Balsara softening, in units of c/H */
} orc_switch_params;

/* Viscosity switch after the density loop: alpha_V(t+dt) and B. */
void orc_switch_visc(int64_t n, const orc_params* p, const orc_switch_params* s,
                     const double* h, const double* u, const double* div_v,
                     const double* div_prev, const double* cx, const double* cy,
                     const double* cz, const double* vsig_prev, const double* av_in,
                     double* av_out, double* B) {
    const double gg = p->gamma * (p->gamma - 1.0);
    for (int64_t i = 0; i < n; ++i) {
        double H = p->eps * h[i];
        double c = sqrt(gg * u[i]);
        double ddiv = (div_v[i] - div_prev[i]) / s->dt;
        double S = H * H * (ddiv < 0.0 ? -ddiv : 0.0);
        double aloc = S > 0.0 ? s->av_max * S / (vsig_prev[i] * vsig_prev[i] + S) : 0.0;
        double a = av_in[i];
        if (aloc >= a) a = aloc;
        else a = aloc + (a - aloc) * exp(-s->ell * c * s->dt / H);
        if (a < s->av_min) a = s->av_min;
        av_out[i] = a;
        double d = fabs(div_v[i]);
        double w = sqrt(cx[i] * cx[i] + cy[i] * cy[i] + cz[i] * cz[i]);
        double den = d + w + s->bal_eps * c / H;
        B[i] = den > 0.0 ? d / den : 0.0;
    }
}

/* alpha_V,ngb,i = max of av_j over j with r_ij < H_i (j = i included). */
int64_t orc_alpha_ngb(int64_t n, const double* x, const double* y, const double* z,
                      double L, const orc_params* p, const double* h, const double* av,
                      double* out) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, p->mode, p->ncell)) return -1;
#pragma omp parallel
    {
        orc_list l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            gather(&g, i, p->eps * h[i], NULL, 0.0, &l);
            double v = av[i];
            for (int64_t q = 0; q < l.n; ++q)
                if (av[l.a[q].j] > v) v = av[l.a[q].j];
            out[i] = v;
        }
        free(l.a);
    }
    grid_free(&g);
    return 0;
}

/* Conduction switch after the gradient loop: alpha_c(t+dt). */
void orc_switch_cond(int64_t n, const orc_params* p, const orc_switch_params* s,
                     const double* h, const double* u, const double* vsig,
                     const double* lapu, const double* av_ngb, const double* ac_in,
                     double* ac_out) {
    for (int64_t i = 0; i < n; ++i) {
        double H = p->eps * h[i];
        double src = u[i] > 0.0 ? s->beta_c * H * lapu[i] / sqrt(u[i]) : 0.0;
        double rate = src - (ac_in[i] - s->ac_min) * vsig[i] / H;
        double a = ac_in[i] + s->dt * rate;
        double amax = s->ac_max * (1.0 - av_ngb[i] / s->av_max);
        if (a > amax) a = amax;
        if (a < s->ac_min) a = s->ac_min;
        ac_out[i] = a;
    }
}

/*
 * Force loop with the switches: the viscosity of orc_force with
 * alpha_ij = (av_i + av_j)/2 (B_i + B_j)/2, plus artificial conduction
 * (Eq. 19-20, 22) in du/dt.  Same pairs as orc_force.
 */
int64_t orc_force_sw(int64_t n, const double* x, const double* y, const double* z,
                     const double* vx, const double* vy, const double* vz,
                     const double* u, const double* m, double L, const orc_params* p,
                     const double* h, const double* rho, const double* f,
                     const double* av, const double* B, const double* ac,
                     int64_t nidx, const int64_t* idx, double* ax, double* ay,
                     double* az, double* dudt, int32_t* nint) {
    orc_grid g;
    if (grid_build(&g, n, x, y, z, L, p->mode, p->ncell)) return -1;
    const double gm1 = p->gamma - 1.0, gg = p->gamma * gm1;
    double* Hs = (double*)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t k = 0; k < n; ++k) Hs[k] = p->eps * h[k];
    double Hmax = max_of(Hs, n);
    int64_t cnt = (idx ? nidx : n);
#pragma omp parallel
    {
        orc_list l = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < cnt; ++k) {
            int64_t i = idx ? idx[k] : k;
            gather(&g, i, Hs[i], Hs, Hmax, &l);
            double Pi = gm1 * rho[i] * u[i];
            double Ai = f[i] * Pi / (rho[i] * rho[i]);
            double ci = sqrt(gg * u[i]);
            double sx = 0, sy = 0, sz = 0, su = 0;
            int32_t c = 0;
            for (int64_t q = 0; q < l.n; ++q) {
                const orc_nb* v = &l.a[q];
                int64_t j = v->j;
                if (j == i) continue;
                c++;
                if (v->r == 0.0) continue;
                double Pj = gm1 * rho[j] * u[j];
                double Aj = f[j] * Pj / (rho[j] * rho[j]);
                double cj = sqrt(gg * u[j]);
                double ex = v->dx / v->r, ey = v->dy / v->r, ez = v->dz / v->r;
                double gi = v->r < Hs[i] ? kdWdr(v->r, h[i], p->eps) : 0.0;
                double gj = v->r < Hs[j] ? kdWdr(v->r, h[j], p->eps) : 0.0;
                double wx = vx[i] - vx[j], wy = vy[i] - vy[j], wz = vz[i] - vz[j];
                double vdote = wx * ex + wy * ey + wz * ez;
                double rsum = rho[i] + rho[j];
                double nu = 0.0;
                if (p->visc) {
                    double mu = vdote < 0.0 ? vdote : 0.0;
                    double vsig = ci + cj - p->beta * mu;
                    double aij = 0.5 * (av[i] + av[j]) * 0.5 * (B[i] + B[j]);
                    nu = -aij * mu * vsig / rsum;
                }
                double fg = f[i] * gi + f[j] * gj;
                double sa = Ai * gi + Aj * gj + 0.5 * nu * fg;
                sx -= m[j] * sa * ex;
                sy -= m[j] * sa * ey;
                sz -= m[j] * sa * ez;
                su += m[j] * vdote * (Ai * gi + 0.25 * nu * fg);
                /* artificial conduction */
                double psum = Pi + Pj;
                double acij = psum > 0.0 ? (Pi * ac[i] + Pj * ac[j]) / psum : 0.0;
                double vc = fabs(vdote) + sqrt(2.0 * fabs(Pi - Pj) / rsum);
                su += acij * vc * m[j] * (u[i] - u[j]) * fg / rsum;
            }
            ax[i] = sx; ay[i] = sy; az[i] = sz; dudt[i] = su;
            if (nint) nint[i] = c;
        }
        free(l.a);
    }
    free(Hs);
    grid_free(&g);
    return 0;
}
