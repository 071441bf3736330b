// Workgroup-level helpers for the control kernels: deterministic reductions
// over a 256-thread block and the per-beam terms of the eq. 2 smoothing.
#pragma once

#include <hip/hip_runtime.h>

namespace vmat {

constexpr int CTRL = 256;  // threads of every control kernel

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block in a fixed tree; every thread gets the result.
__device__ __forceinline__ double bsum(double v, double* sh) {
    v = wave_sum_d(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double bmax(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ double bmin(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
    __syncthreads();
    return r;
}

__device__ __forceinline__ int bor(int v, int* sh) {
    v = __any(v) ? 1 : 0;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const int r = sh[0] | sh[1] | sh[2] | sh[3];
    __syncthreads();
    return r;
}

// Several block reductions in one barrier round.  Each value keeps the tree
// of its single form (bsum, bmax, bmin; an OR as the maximum of 0/1), so the
// results are the same bits as K separate reductions.
enum : int { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2 };

template <int OP>
__device__ __forceinline__ double red_op(double a, double b) {
    return OP == RED_SUM ? a + b : OP == RED_MAX ? fmax(a, b) : fmin(a, b);
}

template <int OP>
__device__ __forceinline__ double red_wave(double v) {
    for (int off = 32; off > 0; off >>= 1) v = red_op<OP>(v, __shfl_down(v, off, 64));
    return v;
}

template <int OP>
__device__ __forceinline__ double red_final(const double* w) {
    return red_op<OP>(red_op<OP>(w[0], w[1]), red_op<OP>(w[2], w[3]));
}

template <int OP0, int OP1>
__device__ __forceinline__ void bred2(double& a, double& b) {
    __shared__ double w[2][CTRL / 64];
    a = red_wave<OP0>(a);
    b = red_wave<OP1>(b);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        w[0][threadIdx.x >> 6] = a;
        w[1][threadIdx.x >> 6] = b;
    }
    __syncthreads();
    a = red_final<OP0>(w[0]);
    b = red_final<OP1>(w[1]);
    __syncthreads();
}

template <int OP0, int OP1, int OP2, int OP3>
__device__ __forceinline__ void bred4(double& a, double& b, double& c, double& d) {
    __shared__ double w[4][CTRL / 64];
    a = red_wave<OP0>(a);
    b = red_wave<OP1>(b);
    c = red_wave<OP2>(c);
    d = red_wave<OP3>(d);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        w[0][threadIdx.x >> 6] = a;
        w[1][threadIdx.x >> 6] = b;
        w[2][threadIdx.x >> 6] = c;
        w[3][threadIdx.x >> 6] = d;
    }
    __syncthreads();
    a = red_final<OP0>(w[0]);
    b = red_final<OP1>(w[1]);
    c = red_final<OP2>(w[2]);
    d = red_final<OP3>(w[3]);
    __syncthreads();
}

// eq. 2 pairs: p < N-1 is (p, p+1); p == N-1 is the wrap pair (N-1, 0) when
// circular.  Returns false when p is not a pair.
__device__ __forceinline__ bool smoothing_pair(int p, int N, int circ, const double* th, int& a, int& b,
                                               double& w) {
    if (p < N - 1) {
        a = p; b = p + 1; w = th[p + 1] - th[p];
        return true;
    }
    if (p == N - 1 && circ && N > 1) {
        a = N - 1; b = 0; w = th[0] + 360.0 - th[N - 1];
        return true;
    }
    return false;
}

__device__ __forceinline__ int n_pairs(int N, int circ) { return N - 1 + ((circ && N > 1) ? 1 : 0); }

// dG/dy_k: the pair ending at k contributes +2(y_k - y_prev)/w, the pair
// starting at k contributes -2(y_next - y_k)/w.
__device__ __forceinline__ double dG_at(int k, const double* y, const double* th, int N, int circ) {
    double tp = 0.0, tn = 0.0;
    if (k > 0) tp = 2.0 * (y[k] - y[k - 1]) / (th[k] - th[k - 1]);
    else if (circ && N > 1) tp = 2.0 * (y[0] - y[N - 1]) / (th[0] + 360.0 - th[N - 1]);
    if (k < N - 1) tn = 2.0 * (y[k + 1] - y[k]) / (th[k + 1] - th[k]);
    else if (circ && N > 1) tn = 2.0 * (y[0] - y[N - 1]) / (th[0] + 360.0 - th[N - 1]);
    return (0.0 + tp) - tn;
}

// G(y) and d^T (Hessian of G) d: this thread's share of the pair sums (the
// _part forms) and the block sums.
__device__ __forceinline__ double smoothing_G_part(const double* y, const double* th, int N, int circ) {
    double s = 0.0;
    for (int p = threadIdx.x; p < n_pairs(N, circ); p += blockDim.x) {
        int a, b;
        double w;
        smoothing_pair(p, N, circ, th, a, b, w);
        const double diff = y[b] - y[a];
        s += diff * diff / w;
    }
    return s;
}

__device__ __forceinline__ double smoothing_dHd_part(const double* d, const double* th, int N, int circ) {
    double s = 0.0;
    for (int p = threadIdx.x; p < n_pairs(N, circ); p += blockDim.x) {
        int a, b;
        double w;
        smoothing_pair(p, N, circ, th, a, b, w);
        const double e = d[b] - d[a];
        s += 2.0 * e * e / w;
    }
    return s;
}

__device__ __forceinline__ double smoothing_G(const double* y, const double* th, int N, int circ, double* sh) {
    return bsum(smoothing_G_part(y, th, N, circ), sh);
}

__device__ __forceinline__ double smoothing_dHd(const double* d, const double* th, int N, int circ, double* sh) {
    return bsum(smoothing_dHd_part(d, th, N, circ), sh);
}

}  // namespace vmat
