// Vector kernels of the staircase-preconditioned GMRES (Krylov acceleration
// of the stair splitting; its use as a preconditioner is the future work the
// Conclusions name).  All vectors are FP64 in the padded layout [L][MP] with
// zero padding, which every kernel here preserves.  Reductions are
// compensated and in a fixed order, so every cycle is bitwise reproducible.
#include "stc_device.h"

namespace stc {

// Apply-state of the Krylov operator T = M^{-1} N: every scale 1, never
// stopped, so a sweep launch on it is the plain linear map.
__global__ void k_kstate_init(DevState *st) {
    for (int k = threadIdx.x; k < kRing; k += blockDim.x) {
        st->inv_sigma[k] = 1.0;
        st->diff[k] = 0.0;
    }
    if (threadIdx.x == 0) {
        st->stop_flag = 0;
        st->status = kDevOk;
        st->stop_sweep = -1;
        st->last_sweep = 0;
        st->residual = 0.0;
        st->x_sum = 0.0;
        st->test_after = 0;
    }
}

// Term e of a dot kernel: MODE 0 x[e] (e^T x), 1 x[e] w[e], 2 |x[e] - w[e]|.
// The product is rounded on its own: fused into the compensated sum's first
// add, it would differ from the copy the compensation term uses.
template <int MODE>
__device__ inline double dot_term(const double *__restrict__ x, const double *__restrict__ w,
                                  size_t e) {
#pragma clang fp contract(off)
    if constexpr (MODE == 0) return x[e];
    else if constexpr (MODE == 1) return x[e] * w[e];
    else return fabs(x[e] - w[e]);
}

// Partial dot products: block (c, v) sums the terms of V[v] and w over chunk
// c of the vector into part[v * G + c].  A thread takes the elements
// e0 + tid, e0 + tid + kWG, ... in that order; four terms are loaded ahead
// of their compensated adds, so four loads per thread are in flight.
template <int MODE>
__global__ __launch_bounds__(kWG) void k_kdot(const double *__restrict__ V, size_t ld,
                                               const double *__restrict__ w, size_t n,
                                               double *__restrict__ part) {
    __shared__ double sh[4 * kWG / 64];
    const int G = gridDim.x, c = blockIdx.x, v = blockIdx.y;
    const size_t chunk = (n + G - 1) / G;
    const size_t e0 = (size_t)c * chunk, e1 = e0 + chunk < n ? e0 + chunk : n;
    const double *x = V + (size_t)v * ld;
    double s = 0.0, sc = 0.0;
    size_t e = e0 + threadIdx.x;
    for (; e + 3 * kWG < e1; e += 4 * kWG) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = dot_term<MODE>(x, w, e + u * kWG);
#pragma unroll
        for (int u = 0; u < 4; ++u) dd_acc(s, sc, t[u]);
    }
    for (; e < e1; e += kWG) dd_acc(s, sc, dot_term<MODE>(x, w, e));
    s = block_sum_dd(s, sc, sh);
    if (threadIdx.x == 0) part[(size_t)v * G + c] = s;
}

// out[v] = fixed-order compensated sum of the G partials of vector v;
// mode 1: out[0] = sqrt of it (a 2-norm from a self dot).
__global__ __launch_bounds__(kWG) void k_kfold(const double *part, int G, double *out, int mode) {
    __shared__ double sh[4 * kWG / 64];
    const int v = blockIdx.x;
    double s = 0.0, sc = 0.0;
    for (int c = threadIdx.x; c < G; c += kWG) dd_acc(s, sc, part[(size_t)v * G + c]);
    s = block_sum_dd(s, sc, sh);
    if (threadIdx.x == 0) out[v] = mode == 1 ? sqrt(s) : s;
}

// w += sign * sum_v h[v] V[v]  (h in device memory; V, h and w disjoint).
// The sum runs over v in order; the V entries of four v are loaded ahead of
// their multiply-adds, so four loads per thread are in flight.
__global__ __launch_bounds__(kWG) void k_kupdate(const double *__restrict__ V, size_t ld, int nv,
                                                  const double *__restrict__ h, double sign,
                                                  double *__restrict__ w, size_t n) {
    for (size_t e = blockIdx.x * (size_t)kWG + threadIdx.x; e < n; e += (size_t)gridDim.x * kWG) {
        double t = 0.0;
        int v = 0;
        for (; v + 4 <= nv; v += 4) {
            double a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = V[(size_t)(v + u) * ld + e];
#pragma unroll
            for (int u = 0; u < 4; ++u) t += h[v + u] * a[u];
        }
        for (; v < nv; ++v) t += h[v] * V[(size_t)v * ld + e];
        w[e] += sign * t;
    }
}

// out = a x + b y
__global__ __launch_bounds__(kWG) void k_kaxpby(double a, const double *x, double b,
                                                 const double *y, double *out, size_t n) {
    for (size_t e = blockIdx.x * (size_t)kWG + threadIdx.x; e < n; e += (size_t)gridDim.x * kWG)
        out[e] = a * x[e] + b * y[e];
}

// out = x / s[0]  (s in device memory)
__global__ __launch_bounds__(kWG) void k_kscale(const double *x, const double *s, double *out,
                                                 size_t n) {
    const double inv = 1.0 / s[0];
    for (size_t e = blockIdx.x * (size_t)kWG + threadIdx.x; e < n; e += (size_t)gridDim.x * kWG)
        out[e] = x[e] * inv;
}

static int stream_groups(size_t n) {
    size_t g = (n + kWG - 1) / kWG;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_kstate_init(DevState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_kstate_init, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_kdots(const double *V, size_t ld, int nv, const double *w, size_t n, double *part,
                        int G, double *out, bool norm, hipStream_t s, bool absdiff) {
    if (nv < 1 || G < 1) return hipErrorInvalidValue;
    if (!w)
        hipLaunchKernelGGL(k_kdot<0>, dim3(G, nv), dim3(kWG), 0, s, V, ld, w, n, part);
    else if (absdiff)
        hipLaunchKernelGGL(k_kdot<2>, dim3(G, nv), dim3(kWG), 0, s, V, ld, w, n, part);
    else
        hipLaunchKernelGGL(k_kdot<1>, dim3(G, nv), dim3(kWG), 0, s, V, ld, w, n, part);
    hipLaunchKernelGGL(k_kfold, dim3(nv), dim3(kWG), 0, s, part, G, out, norm ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_kupdate(const double *V, size_t ld, int nv, const double *h, double sign,
                          double *w, size_t n, hipStream_t s) {
    if (nv < 1) return hipSuccess;
    hipLaunchKernelGGL(k_kupdate, dim3(stream_groups(n)), dim3(kWG), 0, s, V, ld, nv, h, sign, w,
                       n);
    return hipGetLastError();
}

hipError_t launch_kaxpby(double a, const double *x, double b, const double *y, double *out,
                         size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_kaxpby, dim3(stream_groups(n)), dim3(kWG), 0, s, a, x, b, y, out, n);
    return hipGetLastError();
}

hipError_t launch_kscale(const double *x, const double *sdev, double *out, size_t n,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_kscale, dim3(stream_groups(n)), dim3(kWG), 0, s, x, sdev, out, n);
    return hipGetLastError();
}

}  // namespace stc
