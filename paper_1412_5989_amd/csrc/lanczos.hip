// Lowest eigenpair of the Hamiltonian by the Lanczos method on the device
// (the step that follows the construction in a CI run: repeated products of
// H with a vector plus orthogonalization, paper Sec. 1-2).  H is the full
// symmetric matrix in CSR form (both triangles, from the full count / fill
// passes), or the stored upper triangle of the construction itself (half the
// bytes per product, a scatter for the transposed half), FP32 values; vectors
// are FP64.
//
// Kernels: y = H x (one wavefront per row, fixed summation order, so the
// product is reproducible bit for bit), c = V^T w over the Lanczos vectors,
// w -= V c, and the Ritz vector V y.  Each iteration orthogonalizes the new
// vector against all earlier ones twice (classical Gram-Schmidt, repeated),
// which keeps the basis orthogonal to rounding.  The small tridiagonal matrix
// stays on the host: its lowest eigenvalue by bisection on Sturm counts, its
// eigenvector by inverse iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ci_internal.h"

namespace ci {
namespace {

template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> glb(const T* p)
{
    return (gptr<T>)p;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
    // fixed butterfly: every lane ends with the same sum, in the same order
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int kSpmvWaves = 4;

// y[i] = sum_e val[e] x[col[e]] over row i (row_ptr values are positions in
// col / val; col are row indices inside the basis).
__global__ void __launch_bounds__(64 * kSpmvWaves) spmv_kernel(const int64_t* __restrict__ row_ptr,
                                                              const int32_t* __restrict__ col,
                                                              const float* __restrict__ val,
                                                              const double* __restrict__ x, double* __restrict__ y,
                                                              int64_t nrows)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * kSpmvWaves + (threadIdx.x >> 6);
    if (i >= nrows) return;
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    double acc = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += 64) acc += (double)glb(val)[e] * glb(x)[glb(col)[e]];
    acc = wave_sum_f64(acc);
    if (lane == 0) y[i] = acc;
}

// y = H x from the stored upper triangle U alone (row i holds the columns
// j >= i, the diagonal included): y = U x + (U - diag U)^T x.  The row
// product sum_j U_ij x_j is a gather as above; every off-diagonal entry also
// adds U_ij x_i to y_j, a scatter into rows anywhere in the vector, done with
// an FP64 device atomic.  y must be zero at launch (zero_f64 below).  The
// order of the atomics is not fixed, so the product is reproducible to
// rounding only.
__global__ void __launch_bounds__(64 * kSpmvWaves) spmv_upper_kernel(const int64_t* __restrict__ row_ptr,
                                                                    const int32_t* __restrict__ col,
                                                                    const float* __restrict__ val,
                                                                    const double* __restrict__ x,
                                                                    double* __restrict__ y, int64_t nrows)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * kSpmvWaves + (threadIdx.x >> 6);
    if (i >= nrows) return;
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    const double xi = glb(x)[i];
    double acc = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += 64) {
        const int j = glb(col)[e];
        const double v = (double)glb(val)[e];
        acc += v * glb(x)[j];
        if (j != i) atomicAdd(y + j, v * xi);
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) atomicAdd(y + i, acc);
}

__global__ void __launch_bounds__(256) zero_f64(double* __restrict__ y, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = 0.0;
}

constexpr int kDotThreads = 256;
constexpr int kDotBlocks = 128;  // partial sums per vector

// part[k * kDotBlocks + b] = partial sum over block b of V[k][i] * w[i]
__global__ void __launch_bounds__(kDotThreads) multi_dot_partial(const double* __restrict__ V, int64_t ld,
                                                                  const double* __restrict__ w, int64_t n,
                                                                  double* __restrict__ part)
{
    __shared__ double sh[kDotThreads / 64];
    const int k = blockIdx.y;
    const double* v = V + (int64_t)k * ld;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kDotThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kDotThreads)
        acc += glb(v)[i] * glb(w)[i];
    acc = wave_sum_f64(acc);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int t = 0; t < kDotThreads / 64; t++) s += sh[t];
        part[(int64_t)k * gridDim.x + blockIdx.x] = s;
    }
}

// c[k] = sum of the partials of vector k, in block order
__global__ void multi_dot_final(const double* __restrict__ part, int nb, int nv, double* __restrict__ c)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nv) return;
    double s = 0.0;
    for (int b = 0; b < nb; b++) s += part[(int64_t)k * nb + b];
    c[k] = s;
}

// w[i] = alpha * (w[i] - sum_k c[k] V[k][i])   (alpha = 1 for the projection)
__global__ void __launch_bounds__(256) combine_sub(const double* __restrict__ V, int64_t ld, const double* __restrict__ c,
                                                   int nv, double* __restrict__ w, int64_t n, double alpha)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int k = 0; k < nv; k++) s += c[k] * glb(V + (int64_t)k * ld)[i];
        w[i] = alpha * (w[i] - s);
    }
}

// out[i] = scale * sum_k c[k] V[k][i]
__global__ void __launch_bounds__(256) combine(const double* __restrict__ V, int64_t ld, const double* __restrict__ c,
                                               int nv, double* __restrict__ out, int64_t n, double scale)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int k = 0; k < nv; k++) s += c[k] * glb(V + (int64_t)k * ld)[i];
        out[i] = scale * s;
    }
}

// dst = scale * src
__global__ void __launch_bounds__(256) scale_copy(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                                                  double scale)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = scale * src[i];
}

unsigned stream_grid(int64_t n)
{
    const int64_t g = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

// Number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm count).
int sturm_below(const std::vector<double>& a, const std::vector<double>& b, int m, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < m; i++) {
        const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
        q = a[i] - x - (i > 0 ? bb / q : 0.0);
        if (q == 0.0) q = -1e-300;  // just below zero: counted, no division by zero
        if (q < 0.0) cnt++;
    }
    return cnt;
}

// Lowest eigenvalue of the m x m tridiagonal by bisection (to rounding).
double lowest_eig(const std::vector<double>& a, const std::vector<double>& b, int m)
{
    double lo = 0.0, hi = 0.0;
    for (int i = 0; i < m; i++) {  // Gershgorin interval
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = i == 0 ? a[i] - r : std::min(lo, a[i] - r);
        hi = i == 0 ? a[i] + r : std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 4e-16 * std::max(std::fabs(lo), std::fabs(hi)); it++) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_below(a, b, m, mid) >= 1) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Eigenvector of the lowest eigenvalue theta of the tridiagonal by inverse
// iteration, unit norm.  The shift sits just below theta, so T - shift is
// positive definite and the elimination needs no pivoting; each solve
// multiplies the wanted component by about gap / (theta - shift).
std::vector<double> tri_eigvec(const std::vector<double>& a, const std::vector<double>& b, int m, double theta)
{
    const double shift = theta - 1e-10 * std::max(1.0, std::fabs(theta));
    std::vector<double> y(m, 1.0 / std::sqrt((double)m)), d(m), cu(m), z(m);
    for (int it = 0; it < 3; it++) {
        d[0] = a[0] - shift;
        z[0] = y[0] / d[0];
        for (int i = 1; i < m; i++) {
            cu[i - 1] = b[i - 1] / d[i - 1];
            d[i] = (a[i] - shift) - b[i - 1] * cu[i - 1];
            z[i] = (y[i] - b[i - 1] * z[i - 1]) / d[i];
        }
        for (int i = m - 2; i >= 0; i--) z[i] -= cu[i] * z[i + 1];
        double nrm = 0.0;
        for (int i = 0; i < m; i++) nrm += z[i] * z[i];
        nrm = std::sqrt(nrm);
        for (int i = 0; i < m; i++) y[i] = z[i] / nrm;
    }
    return y;
}

}  // namespace

hipError_t launch_spmv(const int64_t* row_ptr, const int32_t* col, const float* val, const double* x, double* y,
                       int64_t nrows, hipStream_t s)
{
    if (nrows > 0)
        hipLaunchKernelGGL(spmv_kernel, dim3((unsigned)((nrows + kSpmvWaves - 1) / kSpmvWaves)),
                           dim3(64 * kSpmvWaves), 0, s, row_ptr, col, val, x, y, nrows);
    return hipGetLastError();
}

hipError_t launch_spmv_upper(const int64_t* row_ptr, const int32_t* col, const float* val, const double* x,
                             double* y, int64_t nrows, hipStream_t s)
{
    if (nrows > 0) {
        hipLaunchKernelGGL(zero_f64, dim3(stream_grid(nrows)), dim3(256), 0, s, y, nrows);
        hipLaunchKernelGGL(spmv_upper_kernel, dim3((unsigned)((nrows + kSpmvWaves - 1) / kSpmvWaves)),
                           dim3(64 * kSpmvWaves), 0, s, row_ptr, col, val, x, y, nrows);
    }
    return hipGetLastError();
}

size_t lanczos_work_bytes(int64_t dim, int max_iter)
{
    const size_t m = (size_t)max_iter + 1;
    return sizeof(double) * (m * (size_t)dim + (size_t)dim + m * kDotBlocks + 2 * m);
}

// Lanczos with full reorthogonalization.  Returns hipSuccess or the first
// HIP error; *eval, *iters and evec (device, unit norm) on success.  upper:
// (row_ptr, col, val) hold the stored upper triangle (symmetric product
// above) instead of the full matrix.
hipError_t run_lanczos(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t D, const double* x0,
                       int max_iter, double tol, double* eval, int* iters, double* evec, void* work, hipStream_t s,
                       bool upper)
{
    double* V = (double*)work;  // [max_iter + 1][D]
    double* w = V + (size_t)(max_iter + 1) * D;
    double* part = w + D;
    double* c = part + (size_t)(max_iter + 1) * kDotBlocks;
    const unsigned g = stream_grid(D);
    const unsigned nbd = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (D + kDotThreads - 1) / kDotThreads));
    std::vector<double> alpha, beta, hc(max_iter + 1);
    hipError_t e = hipSuccess;
    auto dots = [&](const double* Vb, int nv, const double* x) {  // c[0..nv) = Vb^T x, to the host too
        hipLaunchKernelGGL(multi_dot_partial, dim3(nbd, nv), dim3(kDotThreads), 0, s, Vb, (int64_t)D, x, D, part);
        hipLaunchKernelGGL(multi_dot_final, dim3((nv + 63) / 64), dim3(64), 0, s, part, (int)nbd, nv, c);
        e = hipMemcpyAsync(hc.data(), c, sizeof(double) * nv, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    };
    // v0 = x0 / |x0|
    dots(x0, 1, x0);
    if (e != hipSuccess) return e;
    if (!(hc[0] > 0.0)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(scale_copy, dim3(g), dim3(256), 0, s, x0, V, D, 1.0 / std::sqrt(hc[0]));
    double theta = 0.0, prev = 0.0;
    int m = 0;
    for (int j = 0; j < max_iter; j++) {
        double* vj = V + (size_t)j * D;
        e = upper ? launch_spmv_upper(row_ptr, col, val, vj, w, D, s) : launch_spmv(row_ptr, col, val, vj, w, D, s);
        if (e != hipSuccess) return e;
        // two projections against v_0..v_j; alpha_j is the v_j component
        double a = 0.0;
        for (int pass = 0; pass < 2; pass++) {
            dots(V, j + 1, w);
            if (e != hipSuccess) return e;
            a += hc[j];
            hipLaunchKernelGGL(combine_sub, dim3(g), dim3(256), 0, s, V, (int64_t)D, c, j + 1, w, D, 1.0);
        }
        alpha.push_back(a);
        m = j + 1;
        dots(w, 1, w);
        if (e != hipSuccess) return e;
        const double bnorm = std::sqrt(std::max(hc[0], 0.0));
        theta = lowest_eig(alpha, beta, m);
        const bool converged = (j > 0 && std::fabs(theta - prev) <= tol * std::max(1.0, std::fabs(theta))) ||
                               bnorm <= 1e-12 * std::max(1.0, std::fabs(theta)) || m == D;
        prev = theta;
        if (converged || j + 1 == max_iter) break;
        beta.push_back(bnorm);
        hipLaunchKernelGGL(scale_copy, dim3(g), dim3(256), 0, s, w, V + (size_t)(j + 1) * D, D, 1.0 / bnorm);
    }
    // Ritz vector: V y for the tridiagonal eigenvector y
    beta.resize(std::max(m - 1, 0));
    const std::vector<double> y = tri_eigvec(alpha, beta, m, theta);
    e = hipMemcpyAsync(c, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(combine, dim3(g), dim3(256), 0, s, V, (int64_t)D, c, m, evec, D, 1.0);
    dots(evec, 1, evec);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scale_copy, dim3(g), dim3(256), 0, s, evec, evec, D, 1.0 / std::sqrt(hc[0]));
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *eval = theta;
    *iters = m;
    return hipGetLastError();
}

}  // namespace ci
