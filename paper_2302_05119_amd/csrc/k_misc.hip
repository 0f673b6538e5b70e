// Whole-tensor helpers: squared norms, operand conversion to 16-bit types,
// finiteness checks, the direct-residual global fit and the MTTKRP test hook.
#include "dev_common.h"

namespace cpd {

// A kernel that does nothing (one wavefront): the launch-latency floor of a
// sweep is a graph of as many of these as the sweep has kernels.
__global__ __launch_bounds__(64) void k_empty() {}

void launch_empty(hipStream_t q) { hipLaunchKernelGGL(k_empty, dim3(1), dim3(64), 0, q); }

template <typename TS> __device__ __forceinline__ double as_f64(TS x) { return (double)x; }
template <> __device__ __forceinline__ double as_f64<__hip_bfloat16>(__hip_bfloat16 x) { return (double)__bfloat162float(x); }
template <> __device__ __forceinline__ double as_f64<__half>(__half x) { return (double)__half2float(x); }

// Stage 1 of a deterministic sum of squares: workgroup b sums its contiguous range.
template <typename TS>
__global__ __launch_bounds__(256) void k_sqnorm_part(const TS* __restrict__ x, long long n, long long per_block,
                                                     double* __restrict__ part) {
    __shared__ double red[256];
    const long long b0 = blockIdx.x * per_block, b1 = min(n, b0 + per_block);
    double acc = 0.0;
    for (long long i = b0 + threadIdx.x; i < b1; i += 256) {
        const double v = as_f64<TS>(x[i]);
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const double* __restrict__ part, int np, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double acc = 0.0;
    for (int i = 0; i < np; ++i) acc += part[i];
    *out = acc;
}

// Operand copy of a tensor with every row padded to ld elements (zeros), so
// each row starts 16-byte aligned: y[r][c] = x[r][c] for c < I3, else 0.
template <typename TS, typename TD>
__global__ __launch_bounds__(256) void k_pad_copy(const TS* __restrict__ x, TD* __restrict__ y, long long rows, int I3, int ld) {
    const long long n = rows * ld;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const long long r = i / ld;
        const int c = (int)(i % ld);
        y[i] = c < I3 ? (TD)x[r * I3 + c] : (TD)0.0f;
    }
}

template <typename TS>
__global__ __launch_bounds__(256) void k_finite(const TS* __restrict__ x, long long n, int* flag) {
    int bad = 0;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) bad |= !isfinite(as_f64<TS>(x[i]));
    if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// ||M^(s) - [[lambda; U^(1), ..., U^(N)]]||^2 for the slab i1 = blockIdx.x of
// block s (the accepted iterate in slot 1), FP64 accumulation.
template <typename TS, typename T>
__global__ __launch_bounds__(256) void k_resid_slab(const Geo* __restrict__ g, StateP<T> st, const TS* __restrict__ M, int s,
                                                   double* __restrict__ part) {
    __shared__ double red[256];
    __shared__ double w[CPD_MAXR];
    apply_rot(st);
    const int i1 = blockIdx.x;
    const int N = g->N, R = g->R, Rq = g->Rq;
    const T* U1 = st.U[1] + g->uoff[0][s] + (long long)i1 * Rq;
    const double* lam = st.lam[1] + s * Rq;
    if (threadIdx.x < R) w[threadIdx.x] = lam[threadIdx.x] * (double)U1[threadIdx.x];
    __syncthreads();
    double acc = 0.0;
    long long slab = 1;
    for (int m = 1; m < N; ++m) slab *= g->I[s][m];
    const TS* Ms = M + (long long)i1 * slab;
    if (N == 3) {
        const int I2 = g->I[s][1], I3 = g->I[s][2];
        const T* U2 = st.U[1] + g->uoff[1][s];
        const T* U3 = st.U[1] + g->uoff[2][s];
        for (long long e = threadIdx.x; e < (long long)I2 * I3; e += 256) {
            const int i2 = (int)(e / I3), i3 = (int)(e % I3);
            double m = 0.0;
            for (int r = 0; r < R; ++r) m += w[r] * (double)U2[(long long)i2 * Rq + r] * (double)U3[(long long)i3 * Rq + r];
            const double d = as_f64<TS>(Ms[e]) - m;
            acc += d * d;
        }
    } else {
        // order N > 3: the element's row offsets in modes 2 .. N, last mode fastest
        for (long long e = threadIdx.x; e < slab; e += 256) {
            long long off[CPD_MAXN];
            long long x = e;
            for (int m = N - 1; m >= 1; --m) {
                off[m] = g->uoff[m][s] + (x % g->I[s][m]) * Rq;
                x /= g->I[s][m];
            }
            double m = 0.0;
            for (int r = 0; r < R; ++r) {
                double p = w[r];
                for (int q = 1; q < N; ++q) p *= (double)st.U[1][off[q] + r];
                m += p;
            }
            const double d = as_f64<TS>(Ms[e]) - m;
            acc += d * d;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[i1] = red[0];
}

// ---------------------------------------------------------------------------
void launch_sqnorm(const void* src, int dtype, long long n, double* out, double* part, int npart, hipStream_t q) {
    const long long per = (n + npart - 1) / npart;
    if (dtype == 0) hipLaunchKernelGGL(k_sqnorm_part<double>, dim3(npart), dim3(256), 0, q, (const double*)src, n, per, part);
    else if (dtype == 1) hipLaunchKernelGGL(k_sqnorm_part<float>, dim3(npart), dim3(256), 0, q, (const float*)src, n, per, part);
    else if (dtype == 2)
        hipLaunchKernelGGL(k_sqnorm_part<__hip_bfloat16>, dim3(npart), dim3(256), 0, q, (const __hip_bfloat16*)src, n, per, part);
    else hipLaunchKernelGGL(k_sqnorm_part<__half>, dim3(npart), dim3(256), 0, q, (const __half*)src, n, per, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, q, part, npart, out);
}

void launch_pad_copy(const void* src, int src_dtype, void* dst, int dst_dtype, long long rows, int I3, int ld, hipStream_t q) {
    long long nb = (rows * ld + 255) / 256;
    if (nb > 8192) nb = 8192;
    if (nb < 1) nb = 1;
    const dim3 gr((unsigned)nb), bl(256);
    if (src_dtype == 0) hipLaunchKernelGGL((k_pad_copy<double, double>), gr, bl, 0, q, (const double*)src, (double*)dst, rows, I3, ld);
    else if (dst_dtype == 1) hipLaunchKernelGGL((k_pad_copy<float, float>), gr, bl, 0, q, (const float*)src, (float*)dst, rows, I3, ld);
    else if (dst_dtype == 2)
        hipLaunchKernelGGL((k_pad_copy<float, __hip_bfloat16>), gr, bl, 0, q, (const float*)src, (__hip_bfloat16*)dst, rows, I3, ld);
    else hipLaunchKernelGGL((k_pad_copy<float, __half>), gr, bl, 0, q, (const float*)src, (__half*)dst, rows, I3, ld);
}

void launch_finite_check(const void* src, int dtype, long long n, int* flag, hipStream_t q) {
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    if (dtype == 0) hipLaunchKernelGGL(k_finite<double>, dim3((unsigned)nb), dim3(256), 0, q, (const double*)src, n, flag);
    else hipLaunchKernelGGL(k_finite<float>, dim3((unsigned)nb), dim3(256), 0, q, (const float*)src, n, flag);
}

template <typename T>
void launch_resid(const Geo* g, const StateP<T>& st, const void* M, int dtype, int s, int I1, double* part, hipStream_t q) {
    if (dtype == 0) hipLaunchKernelGGL((k_resid_slab<double, T>), dim3(I1), dim3(256), 0, q, g, st, (const double*)M, s, part);
    else hipLaunchKernelGGL((k_resid_slab<float, T>), dim3(I1), dim3(256), 0, q, g, st, (const float*)M, s, part);
}
template void launch_resid<float>(const Geo*, const StateP<float>&, const void*, int, int, int, double*, hipStream_t);
template void launch_resid<double>(const Geo*, const StateP<double>&, const void*, int, int, int, double*, hipStream_t);

void launch_sum_parts(const double* part, int np, double* out, hipStream_t q) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, q, part, np, out);
}

}  // namespace cpd
