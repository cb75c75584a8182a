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
// every key is one contiguous segment.  Passes: count (per key), offsets, fill.
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
// tables that a kernel only reads, read with wavefront-uniform addresses:
// through the constant address space they become scalar loads
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(4))) T* cst(const T* p)
{
    return (const __attribute__((address_space(4))) T*)p;
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

// Work item = (block of kXB consecutive determinants x, key group g): the
// keys are cut into kGroups groups by the position of their first
// determinant, and one wavefront scans the candidates of one group for kXB
// determinants at once (every candidate chunk is loaded once and tested
// against all of them).  The count pass writes the number of partners of each
// x in each key; a per-x scan turns those into segment offsets; the fill pass
// writes each key's records at its offset.
// Sizes from a sweep of the 6Li Nmax = 6 build (determinants per wavefront x
// key groups, 1..16 x 1..16): 2 x 4 gave the shortest step; larger blocks hold
// their determinants in scalar registers that spill, and more groups only add
// wavefronts that scan few candidates each.  On 10B Nmax = 4 (build + count)
// 4 x 4 was within 1 % of it and 4 x 2, 2 x 8 and 8 x 2 were slower.
constexpr int kGroups = 4;
constexpr int kXB = 2;

// keys [k0, k1) of group g: those whose first determinant lies in the g-th slice
__device__ __forceinline__ void key_group(const __attribute__((address_space(4))) int32_t* key_off, int nk,
                                          int nsd, int g, int* k0, int* k1)
{
    const int lo = (int)((int64_t)nsd * g / kGroups), hi = (int)((int64_t)nsd * (g + 1) / kGroups);
    int a = 0, b = 0;
    while (a < nk && key_off[a] < lo) a++;
    b = a;
    while (b < nk && key_off[b] < hi) b++;
    *k0 = a;
    *k1 = b;
}

__device__ __forceinline__ int rank_in(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

template <int W, bool FILL>
__global__ void __launch_bounds__(64 * kPartnerWaves) partner_kernel(PartnerArgs A)
{
    const int lane = threadIdx.x & 63;
    const int item = (int)blockIdx.x * kPartnerWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xb = item / kGroups, g = item - xb * kGroups;
    const int x0 = xb * kXB;
    if (x0 >= A.nsd) return;
    const int nsd = A.nsd;
    const int nx = nsd - x0 < kXB ? nsd - x0 : kXB;  // determinants of this block
    const auto sd = cst(A.sd);
    const auto key_off = cst(A.key_off), key_nq = cst(A.key_nq), key_m2 = cst(A.key_m2);
    int k0, k1;
    key_group(key_off, A.nk, nsd, g, &k0, &k1);
    if (k0 >= k1) return;
    uint64_t xw[kXB][W];
    int mx[kXB], qx[kXB];
    int64_t o1[kXB], o12[kXB];
#pragma unroll
    for (int j = 0; j < kXB; j++) {
        const int x = x0 + (j < nx ? j : 0);
#pragma unroll
        for (int t = 0; t < W; t++) xw[j][t] = sd[(int64_t)x * W + t];
        const int kx = cst(A.sd_key)[x];
        mx[j] = key_m2[kx];
        qx[j] = key_nq[kx];
        o1[j] = FILL ? cst(A.l1_ptr)[x] : 0;
        o12[j] = FILL ? cst(A.l12_ptr)[x] : 0;
    }
    const __attribute__((address_space(1))) uint64_t* col[W];  // word t of every determinant
#pragma unroll
    for (int t = 0; t < W; t++) col[t] = glb(A.sdT) + (int64_t)t * nsd;
    const auto l1 = glbw(A.l1), l12 = glbw(A.l12);
    for (int k = k0; k < k1; k++) {
        const int km = key_m2[k], kq = key_nq[k];
        const int y0 = key_off[k], y1 = key_off[k + 1];
        int c1[kXB], c12[kXB];
        bool same[kXB];
#pragma unroll
        for (int j = 0; j < kXB; j++) {
            same[j] = km == mx[j] && ((kq - qx[j]) & 1) == 0;
            const int64_t sb = (int64_t)(x0 + j) * (A.nk + 1);
            c1[j] = (FILL && j < nx) ? cst(A.seg1)[sb + k] : 0;
            c12[j] = (FILL && j < nx) ? cst(A.seg12)[sb + k] : 0;
        }
        for (int yb = y0; yb < y1; yb += 64) {
            const int y = yb + lane;
            const int yc = y < y1 ? y : y1 - 1;
            uint64_t yw[W];
#pragma unroll
            for (int t = 0; t < W; t++) yw[t] = col[t][yc];
            const bool ok = y < y1;
            // placeholder (x, y); decoded into a partner record afterwards
#pragma unroll
            for (int j = 0; j < kXB; j++) {
                int pc = 0;
#pragma unroll
                for (int t = 0; t < W; t++) pc += __popcll(xw[j][t] ^ yw[t]);
                const bool in1 = ok && j < nx && pc <= 2;
                const bool in12 = ok && j < nx && same[j] && pc <= 4;
                const uint64_t m1 = __ballot(in1), m12 = __ballot(in12);
                if (FILL) {
                    const uint64_t ph = ((uint64_t)(uint32_t)(x0 + j) << 32) | (uint32_t)y;
                    if (in1) l1[o1[j] + c1[j] + rank_in(m1)] = ph;
                    if (in12) l12[o12[j] + c12[j] + rank_in(m12)] = ph;
                }
                c1[j] += __popcll(m1);
                c12[j] += __popcll(m12);
            }
        }
        if (!FILL && lane == 0) {
#pragma unroll
            for (int j = 0; j < kXB; j++)
                if (j < nx) {
                    const int64_t sb = (int64_t)(x0 + j) * (A.nk + 1);
                    glbw(A.seg1)[sb + k] = c1[j];
                    glbw(A.seg12)[sb + k] = c12[j];
                }
        }
    }
}

// One lane per partner: the placeholder (x, y) becomes the partner record
// (local index of y, moved orbits, phase, d).  For l12 also records the
// position of x itself inside its own key segment.
__global__ void __launch_bounds__(256) partner_decode(PartnerArgs A, uint64_t* list, int64_t n, bool is12)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const auto lst = glbw(list);
    const uint64_t ph = lst[t];
    const int x = (int)(ph >> 32), y = (int)(uint32_t)ph;
    const int W = A.W;
    const auto sd = glb(A.sd);
    uint64_t xw[kMaxWords], yw[kMaxWords];
    int pc = 0;
    for (int w = 0; w < kMaxWords; w++) {
        xw[w] = w < W ? sd[(int64_t)x * W + w] : 0;
        yw[w] = w < W ? sd[(int64_t)y * W + w] : 0;
        pc += __popcll(xw[w] ^ yw[w]);
    }
    const int ky = glb(A.sd_key)[y];
    lst[t] = partner_record(xw, yw, W, pc, (uint32_t)(y - glb(A.key_off)[ky]));
    if (is12 && x == y)
        glbw(A.self12)[x] = (int)(t - glb(A.l12_ptr)[x] - glb(A.seg12)[(int64_t)x * (A.nk + 1) + ky]);
}

// Per determinant x: segment counts -> segment offsets (exclusive scan over
// the keys), list lengths into l*_ptr[x + 1].
__global__ void __launch_bounds__(64 * kPartnerWaves) partner_offsets(PartnerArgs A)
{
    const int lane = threadIdx.x & 63;
    const int x = (int)blockIdx.x * kPartnerWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (x >= A.nsd) return;
    const auto s1 = glbw(A.seg1 + (int64_t)x * (A.nk + 1));
    const auto s12 = glbw(A.seg12 + (int64_t)x * (A.nk + 1));
    int run1 = 0, run12 = 0;
    for (int k0 = 0; k0 < A.nk; k0 += 64) {
        const int k = k0 + lane;
        const int a = k < A.nk ? s1[k] : 0, b = k < A.nk ? s12[k] : 0;
        int ia = a, ib = b;
        for (int o = 1; o < 64; o <<= 1) {
            const int ua = __shfl_up(ia, o, 64), ub = __shfl_up(ib, o, 64);
            if (lane >= o) {
                ia += ua;
                ib += ub;
            }
        }
        if (k < A.nk) {
            s1[k] = run1 + ia - a;
            s12[k] = run12 + ib - b;
        }
        run1 += __shfl(ia, 63, 64);
        run12 += __shfl(ib, 63, 64);
    }
    if (lane == 0) {
        s1[A.nk] = run1;
        s12[A.nk] = run12;
        glbw(A.l1_ptr)[x + 1] = run1;
        glbw(A.l12_ptr)[x + 1] = run12;
        if (x == 0) {  // so that the inclusive scan of l*_ptr gives offsets
            glbw(A.l1_ptr)[0] = 0;
            glbw(A.l12_ptr)[0] = 0;
        }
    }
}

}  // namespace

static inline unsigned grid_of(int64_t items) { return (unsigned)((items + kPartnerWaves - 1) / kPartnerWaves); }

template <bool FILL>
static void launch_scan(const PartnerArgs& a, hipStream_t s)
{
    const dim3 g(grid_of((int64_t)((a.nsd + kXB - 1) / kXB) * kGroups)), b(64 * kPartnerWaves);
    switch (a.W) {
        case 1: hipLaunchKernelGGL((partner_kernel<1, FILL>), g, b, 0, s, a); break;
        case 2: hipLaunchKernelGGL((partner_kernel<2, FILL>), g, b, 0, s, a); break;
        case 3: hipLaunchKernelGGL((partner_kernel<3, FILL>), g, b, 0, s, a); break;
        default: hipLaunchKernelGGL((partner_kernel<4, FILL>), g, b, 0, s, a); break;
    }
}

__global__ void partner_no_sd(PartnerArgs A)
{
    glbw(A.l1_ptr)[0] = 0;
    glbw(A.l12_ptr)[0] = 0;
}

hipError_t launch_partner_count(const PartnerArgs& a, hipStream_t s)
{
    if (a.nsd > 0) {
        launch_scan<false>(a, s);
        hipLaunchKernelGGL(partner_offsets, dim3(grid_of(a.nsd)), dim3(64 * kPartnerWaves), 0, s, a);
    } else {
        hipLaunchKernelGGL(partner_no_sd, dim3(1), dim3(1), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_partner_fill(const PartnerArgs& a, int64_t n1, int64_t n12, hipStream_t s)
{
    if (a.nsd > 0) {
        launch_scan<true>(a, s);
        if (n1 > 0)
            hipLaunchKernelGGL(partner_decode, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s, a, a.l1, n1, false);
        if (n12 > 0)
            hipLaunchKernelGGL(partner_decode, dim3((unsigned)((n12 + 255) / 256)), dim3(256), 0, s, a, a.l12, n12, true);
    }
    return hipGetLastError();
}

}  // namespace ci
