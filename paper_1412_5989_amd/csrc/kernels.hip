// HIP kernels of libci for CDNA4 (gfx950): count, scan, fill and adjoint of
// the upper-triangle M-scheme Hamiltonian with a two-body interaction.
//
// Work unit: one wavefront per task = up to 64 consecutive rows that share a
// block (proton key, neutron key) and a proton determinant P; lane l owns row
// (P, N_l).  Every column of such a row is (P', N') with P' a one- or
// two-proton partner of P and N' a partner of N_l (paper Sec. 4.1: for sparse
// chunks, iterate over the quantum-number combinations that can be nonzero).
// The loops over target blocks and over P' are uniform across the wavefront;
// only the innermost loop over N' is per lane.  Columns come out in ascending
// order because blocks, proton partners and neutron partners are each visited
// in ascending order.
//
// The same enumeration (visit_row) drives the count pass, the fill pass and
// the adjoint, so their entry order cannot drift apart.
#include <hip/hip_runtime.h>

#include "ci_internal.h"

namespace ci {

enum { kCount = 0, kFill = 1, kAdjoint = 2 };

__device__ __forceinline__ int rec_d(uint64_t r) { return (int)((r >> 57) & 3); }
__device__ __forceinline__ int rec_local(uint64_t r) { return (int)(r & kRecLocalMask); }
__device__ __forceinline__ int rec_h1(uint64_t r) { return (int)((r >> 24) & 255); }
__device__ __forceinline__ int rec_p1(uint64_t r) { return (int)((r >> 32) & 255); }
__device__ __forceinline__ int rec_h2(uint64_t r) { return (int)((r >> 40) & 255); }
__device__ __forceinline__ int rec_p2(uint64_t r) { return (int)((r >> 48) & 255); }
__device__ __forceinline__ double rec_sign(uint64_t r) { return ((r >> 56) & 1) ? -1.0 : 1.0; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Table position of V_{ab,cd} of class cls (0 pp, 1 pn, 2 nn) with
// species-local orbits (for pn: a, c protons; b, d neutrons).  Returns -1 if
// either pair is outside the stored table; *sg receives the antisymmetry sign.
__device__ __forceinline__ int64_t tb_index(const BasisDev& B, int cls, int a, int b, int c, int d,
                                            double* sg)
{
    double s = 1.0;
    if (cls != 1) {
        if (a > b) { int t = a; a = b; b = t; s = -s; }
        if (c > d) { int t = c; c = d; d = t; s = -s; }
    }
    const int n = B.nsps;
    const uint32_t* P = B.pair + (size_t)cls * n * n;
    const uint32_t e1 = P[a * n + b], e2 = P[c * n + d];
    *sg = s;
    if (e1 == kNoPair || e2 == kNoPair || (e1 >> 16) != (e2 >> 16)) return -1;
    const int sec = (int)(e1 >> 16);
    int64_t r = e1 & 0xffff, q = e2 & 0xffff;
    if (r > q) { int64_t t = r; r = q; q = t; }
    const int64_t ns = B.sec_n[sec];
    return B.sec_off[sec] + r * (2 * ns - r + 1) / 2 + (q - r);
}

// iterate the set orbits of a W-word species determinant
template <typename F>
__device__ __forceinline__ void for_each_orbit(const uint64_t* sd, int W, F f)
{
    for (int w = 0; w < W; w++) {
        uint64_t x = sd[w];
        while (x) {
            const int k = __ffsll((long long)x) - 1;
            x &= x - 1;
            f(w * 64 + k);
        }
    }
}

struct RowCtx {
    const BasisDev* B;
    const float* tbme;  // this basis' table
    double* gacc;       // this basis' FP64 gradient accumulators
    const uint64_t* P;  // proton determinant words (row)
    const uint64_t* N;  // neutron determinant words (row)
};

__device__ __forceinline__ double spe(const BasisDev& B, int orb) { return (B.orb_n[orb] + 1.5) * B.hw; }

// term V_{ab,cd} * coef: returns coef * V for the fill, scatters coef * g for
// the adjoint
template <int MODE>
__device__ __forceinline__ double term(const RowCtx& c, int cls, int a, int b, int cc, int d, double coef,
                                       double g)
{
    double s;
    const int64_t k = tb_index(*c.B, cls, a, b, cc, d, &s);
    if (k < 0) return 0.0;
    if (MODE == kFill) return coef * s * (double)c.tbme[k];
    if (MODE == kAdjoint) atomicAdd(&c.gacc[k], coef * s * g);
    return 0.0;
}

// <P N | H | P N>: single-particle energies + every occupied pair
template <int MODE>
__device__ double diag_element(const RowCtx& c, double g)
{
    const BasisDev& B = *c.B;
    const int W = B.W;
    double v = 0.0;
    for_each_orbit(c.P, W, [&](int a) {
        if (MODE == kFill) v += spe(B, a);
        for_each_orbit(c.P, W, [&](int b) {
            if (b > a) v += term<MODE>(c, 0, a, b, a, b, 1.0, g);
        });
        for_each_orbit(c.N, W, [&](int b) { v += term<MODE>(c, 1, a, b, a, b, 1.0, g); });
    });
    for_each_orbit(c.N, W, [&](int a) {
        if (MODE == kFill) v += spe(B, a);
        for_each_orbit(c.N, W, [&](int b) {
            if (b > a) v += term<MODE>(c, 2, a, b, a, b, 1.0, g);
        });
    });
    return v;
}

// one proton moved (row has p, column has h), neutrons equal:
// phase * [ sum_{k in P, k != p} V_pp(pk, hk) + sum_{b in N} V_pn(pb, hb) ]
template <int MODE>
__device__ double proton_single(const RowCtx& c, uint64_t pr, double g)
{
    const BasisDev& B = *c.B;
    const int h = rec_h1(pr), p = rec_p1(pr);
    const double ph = rec_sign(pr);
    double v = 0.0;
    for_each_orbit(c.P, B.W, [&](int k) {
        if (k != p) v += term<MODE>(c, 0, p, k, h, k, ph, g);
    });
    for_each_orbit(c.N, B.W, [&](int b) { v += term<MODE>(c, 1, p, b, h, b, ph, g); });
    return v;  // the phase is already in each term's coefficient
}

// one neutron moved, protons equal:
// phase * [ sum_{k in N, k != p} V_nn(pk, hk) + sum_{a in P} V_pn(ap, ah) ]
template <int MODE>
__device__ double neutron_single(const RowCtx& c, uint64_t nr, double g)
{
    const BasisDev& B = *c.B;
    const int h = rec_h1(nr), p = rec_p1(nr);
    const double ph = rec_sign(nr);
    double v = 0.0;
    for_each_orbit(c.N, B.W, [&](int k) {
        if (k != p) v += term<MODE>(c, 2, p, k, h, k, ph, g);
    });
    for_each_orbit(c.P, B.W, [&](int a) { v += term<MODE>(c, 1, a, p, a, h, ph, g); });
    return v;  // the phase is already in each term's coefficient
}

// Visit every stored entry of the lane's row in ascending column order.
// COUNT: returns the number of entries.  FILL: writes col/val from pos.
// ADJOINT: reads grad_val from pos and scatters onto the table.
template <int MODE>
__device__ int64_t visit_row(const RowCtx& c, int bi, int ip, int in, bool active, int64_t cap,
                             int64_t pos, int32_t* col, float* val, const float* gval)
{
    const BasisDev& B = *c.B;
    const SpeciesDev& SP = B.sp[0];
    const SpeciesDev& SN = B.sp[1];
    const int kp = B.blk_kp[bi], kn = B.blk_kn[bi];
    const int nkp = SP.nk, nkn = SN.nk;
    const int64_t gP = SP.key_off[kp] + ip;
    const int64_t gN = SN.key_off[kn] + in;
    const uint64_t* P1 = SP.l1 + SP.l1_ptr[gP];
    const uint64_t* P12 = SP.l12 + SP.l12_ptr[gP];
    const int32_t* sP1 = SP.seg1 + gP * (nkp + 1);
    const int32_t* sP12 = SP.seg12 + gP * (nkp + 1);
    const uint64_t* N1 = SN.l1 + SN.l1_ptr[gN];
    const uint64_t* N12 = SN.l12 + SN.l12_ptr[gN];
    const int32_t* sN1 = SN.seg1 + gN * (nkn + 1);
    const int32_t* sN12 = SN.seg12 + gN * (nkn + 1);
    // position of the lane's own determinant inside its key segment of l12
    const int self12 = active ? SN.self12[gN] : 0;
    const int64_t start = pos;
    for (int b2 = bi; b2 < B.nblk; b2++) {
        const int kp2 = B.blk_kp[b2], kn2 = B.blk_kn[b2];
        const bool same_n = (kn2 == kn);
        // proton partners of P in key kp2: all d <= 2 when the neutron key is
        // unchanged, else only d <= 1 (a two-proton move needs N' = N)
        const uint64_t* Ps = same_n ? P12 + sP12[kp2] : P1 + sP1[kp2];
        const int np = same_n ? sP12[kp2 + 1] - sP12[kp2] : sP1[kp2 + 1] - sP1[kp2];
        if (np == 0) continue;
        const int64_t base = B.blk_off[b2];
        const int stride = SN.key_off[kn2 + 1] - SN.key_off[kn2];
        const uint64_t* n1 = N1 + sN1[kn2];
        const int nn1 = active ? sN1[kn2 + 1] - sN1[kn2] : 0;
        const uint64_t* n12 = N12 + sN12[kn2];
        const int nn12 = active ? sN12[kn2 + 1] - sN12[kn2] : 0;
        for (int q = 0; q < np; q++) {
            const uint64_t pr = Ps[q];
            const int dp = rec_d(pr);
            const int ipp = rec_local(pr);
            if (b2 == bi && ipp < ip) continue;  // lower triangle
            const int64_t rowbase = base + (int64_t)ipp * stride;
            if (dp == 2) {
                if (!active) continue;
                // two protons moved, N' = N
                if (MODE == kCount) {
                    pos++;
                } else {
                    if (pos >= cap) break;  // row_ptr inconsistent with this handle
                    double v = 0.0;
                    const double g = (MODE == kAdjoint) ? (double)gval[pos] : 0.0;
                    v = term<MODE>(c, 0, rec_p1(pr), rec_p2(pr), rec_h1(pr), rec_h2(pr),
                                   rec_sign(pr), g);
                    if (MODE == kFill) {
                        col[pos] = (int32_t)(rowbase + in);
                        val[pos] = (float)v;
                    }
                    pos++;
                }
                continue;
            }
            const uint64_t* L = dp == 0 ? n12 : n1;
            const int nl = dp == 0 ? nn12 : nn1;
            const int k0 = (b2 == bi && dp == 0) ? self12 : 0;  // diagonal block: N' >= N
            if (MODE == kCount) {
                pos += (nl > k0) ? nl - k0 : 0;
                continue;
            }
            const int kend = (int)min((int64_t)nl, k0 + (cap - pos));  // stay inside col/val
            for (int k = k0; k < kend; k++) {
                const uint64_t nr = L[k];
                const int dn = rec_d(nr);
                const double g = (MODE == kAdjoint) ? (double)gval[pos] : 0.0;
                double v;
                if (dp == 0) {
                    if (dn == 0) v = diag_element<MODE>(c, g);
                    else if (dn == 1) v = neutron_single<MODE>(c, nr, g);
                    else v = term<MODE>(c, 2, rec_p1(nr), rec_p2(nr), rec_h1(nr), rec_h2(nr),
                                        rec_sign(nr), g);
                } else {  // dp == 1
                    if (dn == 0) v = proton_single<MODE>(c, pr, g);
                    else v = term<MODE>(c, 1, rec_p1(pr), rec_p1(nr), rec_h1(pr), rec_h1(nr),
                                        rec_sign(pr) * rec_sign(nr), g);
                }
                if (MODE == kFill) {
                    col[pos] = (int32_t)(rowbase + rec_local(nr));
                    val[pos] = (float)v;
                }
                pos++;
            }
        }
    }
    return pos - start;
}

template <int MODE>
__global__ void __launch_bounds__(256) row_tile_kernel(const BasisDev* __restrict__ bases,
                                                       const Task* __restrict__ tasks, int64_t ntasks,
                                                       const float* __restrict__ tbme,
                                                       int64_t* __restrict__ row_ptr,
                                                       int32_t* __restrict__ col, float* __restrict__ val,
                                                       const float* __restrict__ gval,
                                                       double* __restrict__ gacc, int64_t nrp)
{
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * (blockDim.x >> 6) + uniform(threadIdx.x >> 6);
    if (t >= ntasks) return;
    const Task tk = tasks[t];
    const BasisDev& B = bases[uniform(tk.basis)];
    const int bi = uniform(tk.block);
    const int kn = B.blk_kn[bi], kp = B.blk_kp[bi];
    const int nKn = B.sp[1].key_off[kn + 1] - B.sp[1].key_off[kn];
    const bool active = lane < uniform(tk.nrows);
    const int r = uniform(tk.r0) + (active ? lane : 0);  // row inside the block
    const int ip = r / nKn, in = r - ip * nKn;
    const int64_t gP = B.sp[0].key_off[kp] + ip;
    const int64_t gN = B.sp[1].key_off[kn] + in;
    RowCtx c;
    c.B = &B;
    c.tbme = tbme ? tbme + B.tbme0 : nullptr;
    c.gacc = gacc ? gacc + B.tbme0 : nullptr;
    c.P = B.sp[0].sd + gP * B.W;
    c.N = B.sp[1].sd + gN * B.W;
    const int64_t i = B.blk_off[bi] + r;
    if (MODE == kCount) {
        const int64_t n = visit_row<kCount>(c, bi, ip, in, active, INT64_MAX, 0, nullptr, nullptr, nullptr);
        if (active) row_ptr[B.row0 + i + 1] = n;
    } else {
        // entries of all bases end at row_ptr[nrp - 1]; no write or read passes it
        const int64_t cap = row_ptr[nrp - 1];
        const int64_t pos = active ? row_ptr[B.row0 + i] : 0;
        visit_row<MODE>(c, bi, ip, in, active, cap, pos, col, val, gval);
    }
}

// ------------------------------------------------------------------ scan
// Inclusive scan of int64 in place, three phases: per-block sums, a single
// block over the block sums, per-block rescan with the carried prefix.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ int64_t block_inclusive_scan(int64_t v, int64_t* sh)
{
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        int64_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    if (lane == 63) sh[wid] = v;
    __syncthreads();
    int64_t add = 0;
    for (int w = 0; w < wid; w++) add += sh[w];
    __syncthreads();
    return v + add;
}

__global__ void __launch_bounds__(kScanThreads) scan_block_sums(const int64_t* __restrict__ x, int64_t n,
                                                                int64_t* __restrict__ sums)
{
    __shared__ int64_t sh[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; k++)
        if (base + k < n) s += x[base + k];
    s = block_inclusive_scan(s, sh);
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kScanThreads) scan_sums_exclusive(int64_t* __restrict__ sums, int64_t nb)
{
    __shared__ int64_t sh[kScanThreads / 64];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int64_t idx = b0 + threadIdx.x;
        const int64_t v = idx < nb ? sums[idx] : 0;
        const int64_t inc = block_inclusive_scan(v, sh);
        const int64_t c0 = carry;
        __syncthreads();
        if (idx < nb) sums[idx] = c0 + inc - v;
        if (threadIdx.x == kScanThreads - 1) carry = c0 + inc;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanThreads) scan_apply(int64_t* __restrict__ x, int64_t n,
                                                           const int64_t* __restrict__ sums)
{
    __shared__ int64_t sh[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t loc[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; k++) {
        loc[k] = base + k < n ? x[base + k] : 0;
        s += loc[k];
    }
    const int64_t inc = block_inclusive_scan(s, sh);
    int64_t run = sums[blockIdx.x] + inc - s;
    for (int k = 0; k < kScanItems; k++) {
        run += loc[k];
        if (base + k < n) x[base + k] = run;
    }
}

// ------------------------------------------------------------------ helpers

__global__ void zero_i64_at(int64_t* __restrict__ x, const int64_t* __restrict__ where, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[where[t]] = 0;
}

__global__ void fill_f64(double* __restrict__ x, int64_t n, double v)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        x[t] = v;
}

__global__ void f64_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        y[t] = (float)x[t];
}

__global__ void nnz_of_bases(const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ first,
                             const int64_t* __restrict__ last, int64_t* __restrict__ nnz, int n)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) nnz[t] = row_ptr[last[t]] - row_ptr[first[t]];
}

// ------------------------------------------------------------------ launchers

static inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_count(const BasisDev* bases, const Task* tasks, int64_t ntasks, int64_t* row_ptr,
                        int64_t nrp, const int64_t* seg_first, int nseg, int64_t* scan_tmp,
                        hipStream_t s)
{
    if (ntasks > 0)
        hipLaunchKernelGGL(row_tile_kernel<kCount>, dim3(grid_for(ntasks, 4)), dim3(256), 0, s, bases,
                           tasks, ntasks, nullptr, row_ptr, nullptr, nullptr, nullptr, nullptr, nrp);
    // the first slot of each basis' segment holds 0 before the scan, so the
    // inclusive scan leaves there the number of entries of the bases before it
    hipLaunchKernelGGL(zero_i64_at, dim3(grid_for(nseg, 256)), dim3(256), 0, s, row_ptr, seg_first, nseg);
    const int64_t nb = (nrp + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nb), dim3(kScanThreads), 0, s, row_ptr, nrp,
                       scan_tmp);
    hipLaunchKernelGGL(scan_sums_exclusive, dim3(1), dim3(kScanThreads), 0, s, scan_tmp, nb);
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, row_ptr, nrp, scan_tmp);
    return hipGetLastError();
}

hipError_t launch_nnz(const int64_t* row_ptr, const int64_t* first, const int64_t* last, int64_t* nnz,
                      int n, hipStream_t s)
{
    hipLaunchKernelGGL(nnz_of_bases, dim3(grid_for(n, 256)), dim3(256), 0, s, row_ptr, first, last, nnz, n);
    return hipGetLastError();
}

hipError_t launch_fill(const BasisDev* bases, const Task* tasks, int64_t ntasks, const float* tbme,
                       const int64_t* row_ptr, int64_t nrp, int32_t* col, float* val, hipStream_t s)
{
    if (ntasks > 0)
        hipLaunchKernelGGL(row_tile_kernel<kFill>, dim3(grid_for(ntasks, 4)), dim3(256), 0, s, bases,
                           tasks, ntasks, tbme, const_cast<int64_t*>(row_ptr), col, val, nullptr,
                           nullptr, nrp);
    return hipGetLastError();
}

hipError_t launch_vjp(const BasisDev* bases, const Task* tasks, int64_t ntasks, const int64_t* row_ptr,
                      int64_t nrp, const float* gval, float* gtbme, double* gacc, int64_t ntbme,
                      hipStream_t s)
{
    if (ntbme > 0)
        hipLaunchKernelGGL(fill_f64, dim3(grid_for(ntbme, 256) < 4096 ? grid_for(ntbme, 256) : 4096),
                           dim3(256), 0, s, gacc, ntbme, 0.0);
    if (ntasks > 0)
        hipLaunchKernelGGL(row_tile_kernel<kAdjoint>, dim3(grid_for(ntasks, 4)), dim3(256), 0, s, bases,
                           tasks, ntasks, nullptr, const_cast<int64_t*>(row_ptr), nullptr, nullptr, gval,
                           gacc, nrp);
    if (ntbme > 0)
        hipLaunchKernelGGL(f64_to_f32, dim3(grid_for(ntbme, 256) < 4096 ? grid_for(ntbme, 256) : 4096),
                           dim3(256), 0, s, gacc, gtbme, ntbme);
    return hipGetLastError();
}

}  // namespace ci
