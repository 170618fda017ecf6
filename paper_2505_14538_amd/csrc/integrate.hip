// integrate.hip -- the leapfrog update between force evaluations: velocities
// and internal energies kicked by the force loop's a and du/dt, positions
// drifted and wrapped into their periodic box.  One thread per particle,
// the caller's arrays in place (no binning needed).
#include "launch.h"

namespace swsph {

template <typename T>
__device__ __forceinline__ T wrap_into(T x, T L) {
    if (x >= L) x -= L;
    if (x < (T)0) x += L;
    // a large step (or rounding of x + L) can still leave [0, L)
    if (!(x >= (T)0 && x < L)) {
        x -= L * floor(x / L);
        if (!(x < L)) x = (T)0;
        if (!(x >= (T)0)) x = (T)0;
    }
    return x;
}

template <typename T>
__global__ void k_kick_drift(int64_t n, T* __restrict__ x, T* __restrict__ y, T* __restrict__ z,
                             T* __restrict__ vx, T* __restrict__ vy, T* __restrict__ vz,
                             T* __restrict__ u, const T* __restrict__ ax,
                             const T* __restrict__ ay, const T* __restrict__ az,
                             const T* __restrict__ dudt, T dtk, T dtd,
                             const int32_t* __restrict__ box_id, int32_t n_box, DriftBoxes boxes) {
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n) return;
    T wx = vx[p], wy = vy[p], wz = vz[p];
    if (dtk != (T)0) {
        wx += ax[p] * dtk;
        wy += ay[p] * dtk;
        wz += az[p] * dtk;
        vx[p] = wx;
        vy[p] = wy;
        vz[p] = wz;
        u[p] += dudt[p] * dtk;
    }
    if (dtd != (T)0) {
        int b = box_id ? box_id[p] : 0;
        b = b < 0 ? 0 : (b >= n_box ? n_box - 1 : b);
        const T L = (T)boxes.L[b];
        x[p] = wrap_into(x[p] + wx * dtd, L);
        y[p] = wrap_into(y[p] + wy * dtd, L);
        z[p] = wrap_into(z[p] + wz * dtd, L);
    }
}

template <typename T>
void launch_kick_drift(int64_t n, void* x, void* y, void* z, void* vx, void* vy, void* vz, void* u,
                       const void* ax, const void* ay, const void* az, const void* dudt,
                       double dt_kick, double dt_drift, const int32_t* box_id, int32_t n_box,
                       const DriftBoxes& boxes, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_kick_drift<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       (T*)x, (T*)y, (T*)z, (T*)vx, (T*)vy, (T*)vz, (T*)u, (const T*)ax,
                       (const T*)ay, (const T*)az, (const T*)dudt, (T)dt_kick, (T)dt_drift,
                       box_id, n_box, boxes);
}
template void launch_kick_drift<float>(int64_t, void*, void*, void*, void*, void*, void*, void*,
                                       const void*, const void*, const void*, const void*, double,
                                       double, const int32_t*, int32_t, const DriftBoxes&,
                                       hipStream_t);
template void launch_kick_drift<double>(int64_t, void*, void*, void*, void*, void*, void*, void*,
                                        const void*, const void*, const void*, const void*,
                                        double, double, const int32_t*, int32_t,
                                        const DriftBoxes&, hipStream_t);

}  // namespace swsph
