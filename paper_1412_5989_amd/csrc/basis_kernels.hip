// Partner lists of the species determinants, built on the device.
//
// For every determinant x of one species (protons or neutrons) the kernel
// scans the candidate determinants y key by key and keeps
//   l1(x):  every y with d(x, y) <= 1 (x itself included), any key;
//   l12(x): every y with d(x, y) <= 2 in the keys of x's 2M and Nq parity,
// where d is half the popcount of x XOR y (the number of moved nucleons).
// For each kept y the moved orbits are decoded with __ffsll (particles in x
// and not in y, holes in y and not in x) and the fermion phase is taken from
// masked popcounts.  Ballot compaction keeps the records in ascending y, so
// every key is one contiguous segment.  Two passes: count, then fill.
#include <hip/hip_runtime.h>

#include "ci_internal.h"

namespace ci {


namespace {

constexpr int kPartnerWaves = 4;

// descriptor pointers are generic; use them through the global address space
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* glb(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* glbw(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

// number of set bits of the W-word string strictly below orbit k
__device__ __forceinline__ int bits_below(const uint64_t* w, int W, int k)
{
    int c = 0;
    for (int t = 0; t < W; t++) {
        const int lo = t * 64;
        if (k >= lo + 64) c += __popcll(w[t]);
        else if (k > lo) c += __popcll(w[t] & ((1ull << (k - lo)) - 1));
    }
    return c;
}

// lowest set orbit of a W-word string (which must have one)
__device__ __forceinline__ int lowest_orbit(const uint64_t* w, int W)
{
    for (int t = 0; t < W; t++)
        if (w[t]) return t * 64 + __ffsll((long long)w[t]) - 1;
    return -1;
}

__device__ __forceinline__ void clear_orbit(uint64_t* w, int k) { w[k >> 6] &= ~(1ull << (k & 63)); }

// Record of partner y (local index yl in its key) of determinant x; pc is the
// popcount of x XOR y (0, 2 or 4).
__device__ uint64_t partner_record(const uint64_t* x, const uint64_t* y, int W, int pc, uint32_t yl)
{
    if (pc == 0) return make_rec(yl, 0, 0, 0, 0, 0, false);
    uint64_t holes[kMaxWords], parts[kMaxWords];
    for (int t = 0; t < kMaxWords; t++) {
        holes[t] = t < W ? (y[t] & ~x[t]) : 0;
        parts[t] = t < W ? (x[t] & ~y[t]) : 0;
    }
    const int h1 = lowest_orbit(holes, W), p1 = lowest_orbit(parts, W);
    if (pc == 2) {
        // orbits of x strictly between the particle and the hole
        const int lo = p1 < h1 ? p1 : h1, hi = p1 < h1 ? h1 : p1;
        const int between = bits_below(x, W, hi) - bits_below(x, W, lo + 1);
        return make_rec(yl, 1, h1, p1, 0, 0, between & 1);
    }
    clear_orbit(holes, h1);
    clear_orbit(parts, p1);
    const int h2 = lowest_orbit(holes, W), p2 = lowest_orbit(parts, W);
    // phase of a+_p1 a+_p2 a_h2 a_h1 on y: T = y without h1, h2 (= x without p1, p2)
    uint64_t T[kMaxWords];
    for (int t = 0; t < kMaxWords; t++) T[t] = t < W ? y[t] : 0;
    clear_orbit(T, h1);
    clear_orbit(T, h2);
    const int e = bits_below(y, W, h1) + bits_below(y, W, h2) - 1 + bits_below(T, W, p1) + bits_below(T, W, p2);
    return make_rec(yl, 2, h1, p1, h2, p2, e & 1);
}

template <bool FILL>
__global__ void __launch_bounds__(64 * kPartnerWaves) partner_kernel(PartnerArgs A)
{
    const int lane = threadIdx.x & 63;
    const int x = (int)blockIdx.x * kPartnerWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (x >= A.nsd) return;
    const int W = A.W;
    uint64_t xw[kMaxWords];
    const auto sd = glb(A.sd);
    const auto key_off = glb(A.key_off), key_nq = glb(A.key_nq), key_m2 = glb(A.key_m2);
    for (int t = 0; t < kMaxWords; t++) xw[t] = t < W ? sd[(int64_t)x * W + t] : 0;
    const int kx = glb(A.sd_key)[x];
    const int mx = key_m2[kx], qx = key_nq[kx];
    int c1 = 0, c12 = 0;
    const int64_t o1 = FILL ? glb(A.l1_ptr)[x] : 0, o12 = FILL ? glb(A.l12_ptr)[x] : 0;
    const auto s1 = glbw(A.seg1 + (int64_t)x * (A.nk + 1));
    const auto s12 = glbw(A.seg12 + (int64_t)x * (A.nk + 1));
    const auto l1 = glbw(A.l1), l12 = glbw(A.l12);
    for (int k = 0; k < A.nk; k++) {
        if (FILL && lane == 0) {
            s1[k] = c1;
            s12[k] = c12;
        }
        const bool same = key_m2[k] == mx && ((key_nq[k] - qx) & 1) == 0;
        const int c12k = c12;  // first l12 record of key k
        const int y0 = key_off[k], y1 = key_off[k + 1];
        for (int yb = y0; yb < y1; yb += 64) {
            const int y = yb + lane;
            int pc = 64;
            uint64_t yw[kMaxWords] = {0, 0, 0, 0};
            if (y < y1) {
                pc = 0;
                for (int t = 0; t < W; t++) {
                    yw[t] = sd[(int64_t)y * W + t];
                    pc += __popcll(xw[t] ^ yw[t]);
                }
            }
            const bool in1 = pc <= 2;
            const bool in12 = same && pc <= 4;
            const uint64_t m1 = __ballot(in1), m12 = __ballot(in12);
            if (FILL && (in1 || in12)) {
                const uint64_t rec = partner_record(xw, yw, W, pc, (uint32_t)(y - y0));
                if (in1) {
                    const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m1 >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m1, 0));
                    l1[o1 + c1 + r] = rec;
                }
                if (in12) {
                    const int r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m12 >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m12, 0));
                    l12[o12 + c12 + r] = rec;
                    if (y == x) glbw(A.self12)[x] = c12 - c12k + r;
                }
            }
            c1 += __popcll(m1);
            c12 += __popcll(m12);
        }
    }
    if (lane == 0) {
        if (FILL) {
            s1[A.nk] = c1;
            s12[A.nk] = c12;
        } else {
            glbw(A.l1_ptr)[x + 1] = c1;
            glbw(A.l12_ptr)[x + 1] = c12;
        }
    }
}

}  // namespace

hipError_t launch_partner_count(const PartnerArgs& a, hipStream_t s)
{
    if (a.nsd > 0)
        hipLaunchKernelGGL(partner_kernel<false>, dim3((a.nsd + kPartnerWaves - 1) / kPartnerWaves),
                           dim3(64 * kPartnerWaves), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_partner_fill(const PartnerArgs& a, hipStream_t s)
{
    if (a.nsd > 0)
        hipLaunchKernelGGL(partner_kernel<true>, dim3((a.nsd + kPartnerWaves - 1) / kPartnerWaves),
                           dim3(64 * kPartnerWaves), 0, s, a);
    return hipGetLastError();
}

}  // namespace ci
