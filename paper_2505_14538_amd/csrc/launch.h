// launch.h -- host-side launch wrappers shared by the library's translation
// units (not part of the C ABI).
#pragma once

#include "swsph_internal.h"

namespace swsph {

// Density task lists reach this factor beyond the largest guessed support of
// their tile (the Newton iteration's room before a fix-up pass).
constexpr double DENS_MARGIN = 1.2;
// The same factor for the single-launch step, whose boxes are redone whole
// when any of their roots lies beyond it (a wider margin pays there).
constexpr double SINGLE_MARGIN = 1.25;

// Events around loop-kernel launches (SWSPH_TIMING); owned by the plan.
struct Timer;
void timer_begin(Timer* t, int loop, hipStream_t s);
void timer_end(Timer* t, int loop, hipStream_t s);

// Scheme constants and options passed to the loop kernels.
struct Scheme {
    double eta, eps, gamma, alpha, beta, h_tol;
    int32_t h_max_iter;
    uint32_t flags;
    int32_t leaf_max;
    int32_t order;  // 0: tiles by decreasing cost, 1: in Morton order
    Timer* timer;   // nullable
};

// Device pointers of one bin (all inside the workspace).
struct BinPtrs {
    Counters* cnt;
    BoxInfo* boxtab;
    uint32_t* keys;
    int32_t *slot, *tmpidx, *perm, *rank;
    int32_t *fine_count, *cstart, *scan_part;
    void *pos4, *vel4, *hs, *dens4;
    float* hmaxpyr;
    Tile* tiles;               // the tile set of the loop at hand
    int32_t* order;
    unsigned long long* ntiles;  // its device count
    Tile* tiles_d;             // density tiles (may alias tiles)
    int32_t* order_d;
    int32_t* dparent;          // gradient/force tile containing each density tile
    int32_t *ord_table, *ord_base;  // cost-order sort: class x block counts, their scan
    int32_t *cand_cnt, *cand_off;
    uint32_t* cands;
    int64_t cand_cap;
    int64_t build_waves;       // most task-build wavefronts (the capacity counts one window each)
    float* trad;
    int32_t* tflag;
    float* fbox;               // density fix-ups: box of each flagged tile's pending
                               // particles (lo xyz, hi xyz)
    float* trad_d;             // single-launch step: density fix-up radii
    int32_t* fredo;            // single-launch step: gradient/force tiles to redo
    int32_t* forder;           // single-launch step: the launch's task order
    uint32_t* boxph;           // single-launch step: per box, done count | redo bit
                               // (32 words apart); then the density tiles of each box;
                               // then each box's smallest gradient/force list radius
    void *d_out, *g_out, *f_out, *adj;
    int32_t *d_int, *f_int;
    int64_t n;
    int32_t n_box;
    int32_t tile;      // most particles per tile (gradient/force)
    int32_t tile_d;    // most particles per density tile
    int64_t tile_cap;  // most tiles (the device holds the count: cnt->n_tiles)
    int64_t n_fine, n_pyr;
};

// Launch modes of the loop kernels.
enum Mode { MODE_QUEUE = 0, MODE_FLAT = 1, MODE_PER_TASK = 2 };

void launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t s);
void launch_copy_u64(unsigned long long* dst, const unsigned long long* src, hipStream_t s);
struct BinPtrs;
BinPtrs density_view(const BinPtrs& b);
template <typename T>
void launch_keys(const swsph_particles* p, const BoxInfo* boxtab, uint32_t* keys,
                 int32_t* slot, int32_t* fine_count, Counters* cnt, hipStream_t s);
int64_t scan_partials_needed(int64_t n);
void launch_exclusive_scan(const int32_t* in, int64_t n, int32_t* part, int32_t* out,
                           hipStream_t s);
void launch_box_check(int32_t n_box, const BoxInfo* boxtab, const int32_t* cstart, Counters* cnt,
                      hipStream_t s);
void launch_scatter_stable(int64_t n, const uint32_t* keys, const int32_t* slot,
                           const int32_t* cstart, int32_t* tmpidx, int32_t* perm,
                           int32_t* rank, Counters* cnt, hipStream_t s);
template <typename T>
void launch_gather(const swsph_particles* p, const BoxInfo* boxtab, const uint32_t* keys,
                   const int32_t* cstart, const int32_t* perm, double eta, void* pos4,
                   void* vel4, void* hs, hipStream_t s);
template <typename T>
void launch_make_tiles(const BinPtrs& b, hipStream_t s);
unsigned wave_grid(int64_t items, int wpb);
// Task-list entries a build wavefront takes from the bump counter at a time
// (its window); the candidate capacity leaves room for one window per
// wavefront that can be resident (32 per CU).
constexpr int64_t TASK_CHUNK = 8192;
constexpr int64_t BUILD_WAVES_PER_CU = 32;
template <typename T>
void launch_unsort(int64_t n, const int32_t* rank, const void* in, void* out, hipStream_t s);
// Up to 12 binned arrays of one type back to the caller's order in one launch.
struct UnsortSet {
    const void* in[12];
    void* out[12];
    int k;
};
template <typename T>
void launch_unsort_multi(int64_t n, const int32_t* rank, const UnsortSet& set, hipStream_t s);
template <typename T>
void launch_sortcopy(int64_t n, const int32_t* perm, const void* in, void* out, hipStream_t s);

// tasks.hip: mode 0 density, 1 gradient, 2 force, 3 force at the density
// margin over the guessed supports (single-launch step); fixup: only the
// listed tiles (density: flagged for a fix-up; force: to redo)
template <typename T>
void launch_tasks(const BinPtrs& b, const Scheme& sc, int mode, bool fixup, hipStream_t s);
void launch_order(const BinPtrs& b, hipStream_t s);
int64_t order_table_size(int64_t tile_cap);

// loops.hip
template <typename T>
int launch_density(const BinPtrs& b, const Scheme& sc, int mode, int lds_cap, hipStream_t s);
template <typename T>
void launch_prep_dens(const BinPtrs& b, const Scheme& sc, const swsph_density_out* d,
                      hipStream_t s);
template <typename T>
void launch_hmax_pyramid(const BinPtrs& b, const Scheme& sc, hipStream_t s);
// The task lists of the loop below (build first).
template <typename T>
void launch_gf_tasks(const BinPtrs& b, const Scheme& sc, hipStream_t s);
// The gradient and the force loop in one kernel (binned outputs g_out, f_out).
template <typename T>
int launch_force(const BinPtrs& b, const Scheme& sc, int mode, int lds_cap, hipStream_t s);
// Constants of the time-dependent switches (swsph_switch_params).
struct SwitchConsts {
    double dt, av_max, av_min, ell, beta_c, ac_min, ac_max, bal_eps;
};
// The gradient and force loops with the switches (lists from launch_gf_tasks).
template <typename T>
int launch_switch_loops(const BinPtrs& b, const Scheme& sc, const SwitchConsts& sw,
                        const swsph_density_out* d, const swsph_switch_state* st, int mode,
                        int lds_cap, hipStream_t s);
// The single-launch step's loops (after the bin): lists at the margin over
// the guessed supports, one launch for every box's density, gradient and
// force tiles, then the separate-launch path for what it left (the binned
// outputs as after launch_density and launch_force).
template <typename T>
int launch_single(const BinPtrs& b, const Scheme& sc, int lds_cap_d, int lds_cap, hipStream_t s);
template <typename T>
int launch_backward(const BinPtrs& b, const Scheme& sc, const swsph_force_grad* g,
                    const swsph_density_out* d, int lds_cap, hipStream_t s);
int device_cu_count();

// integrate.hip: the leapfrog kick (v += a dt_kick, u += du/dt dt_kick) and
// drift (x += v dt_drift, wrapped into the particle's box)
constexpr int DRIFT_MAX_BOXES = 64;
struct DriftBoxes {
    double L[DRIFT_MAX_BOXES];
};
template <typename T>
void launch_kick_drift(int64_t n, void* x, void* y, void* z, void* vx, void* vy, void* vz, void* u,
                       const void* ax, const void* ay, const void* az, const void* dudt,
                       double dt_kick, double dt_drift, const int32_t* box_id, int32_t n_box,
                       const DriftBoxes& boxes, hipStream_t s);

}  // namespace swsph
