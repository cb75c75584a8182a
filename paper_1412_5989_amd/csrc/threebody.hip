// Three-body basis transformation (paper Sec. 3): m-scheme matrix elements of
// a three-body interaction, decoupled on request from its coupled-JT form.
//
// Coupled basis: ordered triples (a, b, c) of oscillator orbitals (n, l, j)
// with N_a + N_b + N_c <= N3max, coupled as ((j_a j_b) J_ab, j_c) J and
// ((1/2 1/2) T_ab, 1/2) T.  The interaction is diagonal in J and T and
// independent of their projections, so the input A is a set of dense blocks,
// one per (bra triple, ket triple, J, T), over the channels (J_ab, T_ab) x
// (J_de, T_de).  The blocks are stored in the order the decoupling loops read
// them: triple pair, then J ascending, then T, then row-major channels
// (paper Sec. 3.1: only potentially nonzero elements are kept, in loop order).
//
// A request is six m-scheme orbits (a b c | d e f) (species-combined index:
// proton orbit k -> k, neutron k -> n_sps + k; isospin projection +1/2 for a
// proton).  Its element is sum over J_ab, J_de, J, T_ab, T_de, T of the
// Clebsch-Gordan coefficients of bra and ket times the coupled element; one
// request per lane (paper Sec. 3.2: one element per thread; the loop bounds
// depend on the request).  FP32 input, FP64 sums, FP32 output.
#include "threebody.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ci_internal.h"

namespace ci {

namespace {

__host__ __device__ __forceinline__ int iabs(int x) { return x < 0 ? -x : x; }

__host__ __device__ __forceinline__ bool triangle2(int a2, int b2, int c2)
{
    return iabs(a2 - b2) <= c2 && c2 <= a2 + b2 && ((a2 + b2 + c2) & 1) == 0;
}

// Range of the intermediate J_ab (doubled, step 2) of a triple with orbit
// spins ja, jb, jc coupled to J: J_ab runs over [|ja - jb|, ja + jb] and must
// close a triangle with jc and J; returns the count, *lo the first value.
__host__ __device__ __forceinline__ int jab_range(int ja, int jb, int jc, int J, int* lo)
{
    const int l = max(iabs(ja - jb), iabs(J - jc)), h = min(ja + jb, J + jc);
    *lo = l;
    return h >= l ? (h - l) / 2 + 1 : 0;
}

// (J_ab, T_ab) channels of the triple coupled to (J, T): T_ab in {0, 1} for
// T = 1/2 and T_ab = 1 for T = 3/2, J_ab in its range, J_ab-major.
__host__ __device__ __forceinline__ int n_channels(int ja, int jb, int jc, int J, int T)
{
    int lo;
    return jab_range(ja, jb, jc, J, &lo) * (T == 1 ? 2 : 1);
}

// <j1 m1 j2 m2 | J M> (doubled arguments) by the Racah formula, in long
// double; host only, for the tables.
double racah_cg(int j1, int m1, int j2, int m2, int J, int M)
{
    if (m1 + m2 != M || iabs(m1) > j1 || iabs(m2) > j2 || iabs(M) > J) return 0.0;
    if (((j1 + m1) & 1) || ((j2 + m2) & 1) || ((J + M) & 1) || !triangle2(j1, j2, J)) return 0.0;
    static const std::vector<long double> f = [] {
        std::vector<long double> t(200, 1.0L);
        for (int k = 1; k < 200; k++) t[k] = t[k - 1] * k;
        return t;
    }();
    const int a = (j1 + j2 - J) / 2, b = (j1 - j2 + J) / 2, c = (-j1 + j2 + J) / 2, d = (j1 + j2 + J) / 2 + 1;
    const long double pre = sqrtl((long double)(J + 1) * f[a] * f[b] * f[c] / f[d] * f[(J + M) / 2] *
                                  f[(J - M) / 2] * f[(j1 - m1) / 2] * f[(j1 + m1) / 2] * f[(j2 - m2) / 2] *
                                  f[(j2 + m2) / 2]);
    const int e1 = (j1 - m1) / 2, e2 = (j2 + m2) / 2, e3 = (J - j2 + m1) / 2, e4 = (J - j1 - m2) / 2;
    const int kmin = std::max({0, -e3, -e4}), kmax = std::min({a, e1, e2});
    long double sum = 0.0L;
    for (int k = kmin; k <= kmax; k++) {
        const long double t = 1.0L / (f[k] * f[a - k] * f[e1 - k] * f[e2 - k] * f[e3 + k] * f[e4 + k]);
        sum += (k & 1) ? -t : t;
    }
    return (double)(pre * sum);
}

// table entry counts of one (j1, j2) pair
int cg_block(int j1, int j2) { return (j1 + 1) * (j2 + 1) * (std::min(j1, j2) + 1); }

void build_cg_tables(int nj, std::vector<int32_t>& off1, std::vector<float>& cg1, std::vector<int32_t>& off2,
                     std::vector<float>& cg2)
{
    const int jmax = 2 * nj - 1;
    off1.assign((size_t)nj * nj, 0);
    cg1.clear();
    for (int a = 0; a < nj; a++)
        for (int b = 0; b < nj; b++) {
            const int j1 = 2 * a + 1, j2 = 2 * b + 1, nJ = std::min(j1, j2) + 1;
            off1[(size_t)a * nj + b] = (int32_t)cg1.size();
            for (int m1 = -j1; m1 <= j1; m1 += 2)
                for (int m2 = -j2; m2 <= j2; m2 += 2)
                    for (int i = 0; i < nJ; i++)
                        cg1.push_back((float)racah_cg(j1, m1, j2, m2, iabs(j1 - j2) + 2 * i, m1 + m2));
        }
    off2.assign((size_t)(jmax + 1) * nj, 0);
    cg2.clear();
    for (int A = 0; A <= jmax; A++)
        for (int c = 0; c < nj; c++) {
            const int J12 = 2 * A, j3 = 2 * c + 1, nJ = std::min(J12, j3) + 1;
            off2[(size_t)A * nj + c] = (int32_t)cg2.size();
            for (int M12 = -J12; M12 <= J12; M12 += 2)
                for (int m3 = -j3; m3 <= j3; m3 += 2)
                    for (int i = 0; i < nJ; i++)
                        cg2.push_back((float)racah_cg(J12, M12, j3, m3, iabs(J12 - j3) + 2 * i, M12 + m3));
        }
}

// Coefficient lookups; the offset tables of both coupling steps sit in LDS
// (off1: [nj][nj], off2: [2 nj][nj]).
struct CgView {
    const int* off1;
    const int* off2;
    const float* cg1;
    const float* cg2;
    int nj;
};

// <j1 m1 j2 m2 | J, m1 + m2> for odd j1, j2; J must close the triangle and
// |m1 + m2| <= J must hold (the table index assumes both).
__device__ __forceinline__ float cg_first(const CgView& C, int j1, int m1, int j2, int m2, int J)
{
    const int base = C.off1[((j1 - 1) >> 1) * C.nj + ((j2 - 1) >> 1)];
    return C.cg1[base + (((m1 + j1) >> 1) * (j2 + 1) + ((m2 + j2) >> 1)) * (min(j1, j2) + 1) + ((J - iabs(j1 - j2)) >> 1)];
}

// <J12 M12 j3 m3 | J, M12 + m3> for even J12, odd j3; |M12| <= J12 and the
// triangle (J12, j3, J) must hold.
__device__ __forceinline__ float cg_second(const CgView& C, int J12, int M12, int j3, int m3, int J)
{
    const int base = C.off2[(J12 >> 1) * C.nj + ((j3 - 1) >> 1)];
    return C.cg2[base + (((M12 + J12) >> 1) * (j3 + 1) + ((m3 + j3) >> 1)) * (min(J12, j3) + 1) +
                 ((J - iabs(J12 - j3)) >> 1)];
}

// Isospin part of a triple's coefficient: <1/2 t1 1/2 t2 | T_ab, t1 + t2>
// <T_ab, t1 + t2, 1/2 t3 | T, MT> for (T, T_ab) = (1/2, 0), (1/2, 1), (3/2, 1).
__device__ __forceinline__ void iso_coeffs(const CgView& C, int t1, int t2, int t3, float c[3])
{
    const int MTab = t1 + t2;
    const float c0 = MTab == 0 ? cg_first(C, 1, t1, 1, t2, 0) * cg_second(C, 0, 0, 1, t3, 1) : 0.0f;
    const float c1 = cg_first(C, 1, t1, 1, t2, 2);
    const int MT = MTab + t3;
    c[0] = (MT == 1 || MT == -1) ? c0 : 0.0f;
    c[1] = (MT == 1 || MT == -1) ? c1 * cg_second(C, 2, MTab, 1, t3, 1) : 0.0f;
    c[2] = c1 * cg_second(C, 2, MTab, 1, t3, 3);
}

constexpr int kDecoupleThreads = 64;
constexpr int kBraRows = 16;  // compacted bra rows per pass over the ket columns

__host__ __device__ constexpr size_t decouple_lds_bytes(int nj)
{
    return (size_t)kBraRows * kDecoupleThreads * 5 + (size_t)3 * nj * nj * 4;
}

// One request per lane (paper Sec. 3.2: the loop bounds depend on the
// request).  Per (J, T) block the bra coefficients that do not vanish are
// compacted into this lane's LDS column (value, row), up to kBraRows at a
// time; the ket loop then reads only rows and columns with nonzero
// coefficients.  With an order, lane r works on request order[r].
__global__ void __launch_bounds__(kDecoupleThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) decouple_kernel(ThreeBodyDev T, const float* __restrict__ A,
                                                                    const int32_t* __restrict__ req, int64_t n,
                                                                    const int32_t* __restrict__ order,
                                                                    float* __restrict__ out)
{
    extern __shared__ unsigned char smem[];
    float* cb = (float*)smem;                                            // [kBraRows][kDecoupleThreads]
    unsigned char* rb = smem + (size_t)kBraRows * kDecoupleThreads * 4;  // [kBraRows][kDecoupleThreads]
    int* offs = (int*)(smem + (size_t)kBraRows * kDecoupleThreads * 5);
    const int lane = threadIdx.x;
    const int nj = T.nj, n1 = nj * nj;
    for (int i = lane; i < 3 * n1; i += kDecoupleThreads) offs[i] = i < n1 ? T.cg1_off[i] : T.cg2_off[i - n1];
    __syncthreads();
    const CgView C{offs, offs + n1, T.cg1, T.cg2, nj};
    const int64_t g = (int64_t)blockIdx.x * kDecoupleThreads + lane;
    if (g >= n) return;
    const int64_t r = order ? (int64_t)order[g] : g;
    int o[6];
    bool ok = true;
    for (int k = 0; k < 6; k++) {
        o[k] = req[r * 6 + k];
        ok = ok && o[k] >= 0 && o[k] < 2 * T.nsps;
    }
    double sum = 0.0;
    if (ok) {
        int al[6], m[6], tz[6], j[6], l[6];
        for (int k = 0; k < 6; k++) {
            const int s = o[k] >= T.nsps;
            const uint32_t w = T.orb[o[k] - s * T.nsps];
            al[k] = (int)(w & 0xff);
            j[k] = (int)((w >> 8) & 0xff);
            m[k] = (int)((w >> 16) & 0xff) - 64;
            l[k] = (int)(w >> 24);
            tz[k] = s ? -1 : 1;
        }
        const int M = m[0] + m[1] + m[2], MT = tz[0] + tz[1] + tz[2];
        const int parb = (l[0] + l[1] + l[2]) & 1;
        const int park = (l[3] + l[4] + l[5]) & 1;
        const int n2 = T.nlj * T.nlj;
        const int tb = T.tidx[al[0] * n2 + al[1] * T.nlj + al[2]];
        const int tk = T.tidx[al[3] * n2 + al[4] * T.nlj + al[5]];
        if (M == m[3] + m[4] + m[5] && MT == tz[3] + tz[4] + tz[5] && parb == park && tb >= 0 && tk >= 0) {
            const float* blk = A + T.block_off[(int64_t)tb * T.ntrip + tk];
            float ib[3], ik[3];
            iso_coeffs(C, tz[0], tz[1], tz[2], ib);
            iso_coeffs(C, tz[3], tz[4], tz[5], ik);
            const int Jmax = min(j[0] + j[1] + j[2], j[3] + j[4] + j[5]);
            const int Mab = m[0] + m[1], Mde = m[3] + m[4];
            for (int J = 1; J <= Jmax; J += 2) {
                int lob, lok;
                const int nja = jab_range(j[0], j[1], j[2], J, &lob), njd = jab_range(j[3], j[4], j[5], J, &lok);
                if (nja == 0 || njd == 0) continue;
                const bool mok = M <= J && -M <= J;
                for (int TT = 1; TT <= 3; TT += 2) {
                    const int nt = TT == 1 ? 2 : 1, nk = njd * nt;
                    if (mok && (MT <= TT && -MT <= TT)) {
                        // sum over the nonzero ket columns of the compacted bra rows
                        auto ket_pass = [&](int nz) {
                            double part = 0.0;
                            for (int d = 0; d < njd; d++) {
                                const int jde = lok + 2 * d;
                                if (Mde > jde || -Mde > jde) continue;
                                const float cj = cg_first(C, j[3], m[3], j[4], m[4], jde) *
                                                 cg_second(C, jde, Mde, j[5], m[5], J);
                                for (int t = 0; t < nt; t++) {
                                    const float c = cj * ik[TT == 1 ? t : 2];
                                    if (c == 0.0f) continue;
                                    const float* col = blk + d * nt + t;
                                    double acc = 0.0;
                                    for (int i = 0; i < nz; i++)
                                        acc += (double)cb[i * kDecoupleThreads + lane] *
                                               (double)col[(int)rb[i * kDecoupleThreads + lane] * nk];
                                    part += (double)c * acc;
                                }
                            }
                            return part;
                        };
                        int nz = 0;
                        for (int a = 0; a < nja; a++) {
                            const int jab = lob + 2 * a;
                            if (Mab > jab || -Mab > jab) continue;
                            const float cj = cg_first(C, j[0], m[0], j[1], m[1], jab) *
                                             cg_second(C, jab, Mab, j[2], m[2], J);
                            for (int t = 0; t < nt; t++) {
                                const float c = cj * ib[TT == 1 ? t : 2];
                                if (c == 0.0f) continue;
                                cb[nz * kDecoupleThreads + lane] = c;
                                rb[nz * kDecoupleThreads + lane] = (unsigned char)(a * nt + t);
                                if (++nz == kBraRows) {
                                    sum += ket_pass(nz);
                                    nz = 0;
                                }
                            }
                        }
                        if (nz > 0) sum += ket_pass(nz);
                    }
                    blk += (int64_t)nja * nt * nk;
                }
            }
        }
    }
    out[r] = (float)sum;
}

// ------------------------------------------------------------ request order
//
// Requests differ in cost by two orders of magnitude, and a wavefront runs as
// long as its slowest lane.  An optional counting sort groups them by an
// estimate of their cost (the elements of the (J, T) blocks they read, in
// quarter-octave bins) and hands out the most expensive first.

constexpr int kCostBins = 64;
constexpr int kCostReplicas = 32;  // counters per bin, by workgroup, so that few workgroups share one
constexpr int kCounters = kCostBins * kCostReplicas;
constexpr int kOrderThreads = 256;
constexpr int kOrderPerThread = 4;
constexpr int kOrderPerBlock = kOrderThreads * kOrderPerThread;

// bin of a request from its six orbits' packed words (w[k] = 0 marks an
// index outside [0, 2 n_sps), which costs nothing); tz from the species
__device__ __forceinline__ int cost_bin(const uint32_t w[6], const int tz[6])
{
    int j[6], m[6];
    for (int k = 0; k < 6; k++) {
        if (w[k] == 0u) return 0;
        j[k] = (int)((w[k] >> 8) & 0xff);
        m[k] = (int)((w[k] >> 16) & 0xff) - 64;
    }
    const int M = iabs(m[0] + m[1] + m[2]), MT = iabs(tz[0] + tz[1] + tz[2]);
    const int Jmax = min(j[0] + j[1] + j[2], j[3] + j[4] + j[5]);
    unsigned cost = 0;
    for (int J = M | 1; J <= Jmax; J += 2) {
        int lo;
        const unsigned e = (unsigned)(jab_range(j[0], j[1], j[2], J, &lo) * jab_range(j[3], j[4], j[5], J, &lo));
        cost += e + (MT <= 1 ? 4 * e : 0);
    }
    const unsigned x = cost + 1;
    const int ex = 31 - __builtin_clz(x);
    const int frac = ex >= 2 ? (int)((x >> (ex - 2)) & 3) : (int)((x << (2 - ex)) & 3);
    return min(kCostBins - 1, 4 * ex + frac);
}

// counters: [kCostBins][kCostReplicas] counts, then the same layout of cursors
__global__ void __launch_bounds__(1024) order_clear(uint32_t* counters)
{
    for (int i = threadIdx.x; i < kCounters; i += 1024) counters[i] = 0;
}

__global__ void __launch_bounds__(kOrderThreads) order_histogram(ThreeBodyDev T, const int32_t* __restrict__ req,
                                                                 int64_t n, uint8_t* __restrict__ bin,
                                                                 uint32_t* __restrict__ counts)
{
    __shared__ uint32_t h[kCostBins];
    if (threadIdx.x < kCostBins) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t g0 = (int64_t)blockIdx.x * kOrderPerBlock + threadIdx.x;
    // all loads of the thread's requests first, so that their latencies overlap
    int32_t o[kOrderPerThread][6];
#pragma unroll
    for (int u = 0; u < kOrderPerThread; u++) {
        const int64_t g = g0 + u * kOrderThreads;
#pragma unroll
        for (int k = 0; k < 6; k++) o[u][k] = g < n ? req[g * 6 + k] : -1;
    }
    uint32_t w[kOrderPerThread][6];
    int tz[kOrderPerThread][6];
#pragma unroll
    for (int u = 0; u < kOrderPerThread; u++)
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const int x = o[u][k], s = x >= T.nsps;
            const bool in = x >= 0 && x < 2 * T.nsps;
            w[u][k] = in ? T.orb[x - s * T.nsps] : 0u;  // a packed word is never 0 (2m + 64 > 0)
            tz[u][k] = s ? -1 : 1;
        }
#pragma unroll
    for (int u = 0; u < kOrderPerThread; u++) {
        const int64_t g = g0 + u * kOrderThreads;
        if (g < n) {
            const int b = cost_bin(w[u], tz[u]);
            bin[g] = (uint8_t)b;
            atomicAdd(&h[b], 1u);
        }
    }
    __syncthreads();
    const int rep = blockIdx.x % kCostReplicas;
    if (threadIdx.x < kCostBins && h[threadIdx.x])
        atomicAdd(&counts[threadIdx.x * kCostReplicas + rep], h[threadIdx.x]);
}

// cursors in the order (bin descending, replica ascending): exclusive sums of
// the counts, one workgroup, eight counters per thread
__global__ void __launch_bounds__(256) order_starts(uint32_t* counters)
{
    constexpr int kPer = kCounters / 256;
    __shared__ uint32_t part[256];
    const int t = threadIdx.x;
    uint32_t v[kPer], run = 0;
    for (int i = 0; i < kPer; i++) {
        const int q = t * kPer + i;  // position in the output order
        const int b = kCostBins - 1 - q / kCostReplicas, rep = q % kCostReplicas;
        v[i] = counters[b * kCostReplicas + rep];
        run += v[i];
    }
    part[t] = run;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const uint32_t x = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    run = part[t] - run;  // exclusive prefix of this thread's first counter
    for (int i = 0; i < kPer; i++) {
        const int q = t * kPer + i;
        const int b = kCostBins - 1 - q / kCostReplicas, rep = q % kCostReplicas;
        counters[kCounters + b * kCostReplicas + rep] = run;
        run += v[i];
    }
}

__global__ void __launch_bounds__(kOrderThreads) order_scatter(const uint8_t* __restrict__ bin, int64_t n,
                                                               uint32_t* __restrict__ cursor,
                                                               int32_t* __restrict__ order)
{
    __shared__ uint32_t h[kCostBins];
    __shared__ uint32_t base[kCostBins];
    if (threadIdx.x < kCostBins) h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t g0 = (int64_t)blockIdx.x * kOrderPerBlock + threadIdx.x;
    int b[kOrderPerThread];
    uint32_t rank[kOrderPerThread];
#pragma unroll
    for (int u = 0; u < kOrderPerThread; u++) {
        const int64_t g = g0 + u * kOrderThreads;
        b[u] = g < n ? bin[g] : 0;
    }
#pragma unroll
    for (int u = 0; u < kOrderPerThread; u++)
        rank[u] = g0 + u * kOrderThreads < n ? atomicAdd(&h[b[u]], 1u) : 0u;
    __syncthreads();
    const int rep = blockIdx.x % kCostReplicas;
    if (threadIdx.x < kCostBins && h[threadIdx.x])
        base[threadIdx.x] = atomicAdd(&cursor[threadIdx.x * kCostReplicas + rep], h[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kOrderPerThread; u++) {
        const int64_t g = g0 + u * kOrderThreads;
        if (g < n) order[base[b[u]] + rank[u]] = (int32_t)g;
    }
}

}  // namespace

double clebsch_gordan2(int j1, int m1, int j2, int m2, int J, int M) { return racah_cg(j1, m1, j2, m2, J, M); }

// ------------------------------------------------------------------ host layout

int threebody_plan(int n1max, int n3max, ThreeBodyHost& h, std::string& err)
{
    if (n1max < 0 || n3max < 0 || n1max > 12 || n3max > 3 * n1max) {
        err = "need 0 <= n1max <= 12 and 0 <= n3max <= 3 n1max";
        return CI_EINVAL;
    }
    h.n1max = n1max;
    h.n3max = n3max;
    for (int N = 0; N <= n1max; N++)
        for (int l = N % 2; l <= N; l += 2)
            for (int j2 : {2 * l - 1, 2 * l + 1}) {
                if (j2 < 0) continue;
                const int alpha = (int)h.nlj_N.size();
                h.nlj_N.push_back(N);
                h.nlj_l.push_back(l);
                h.nlj_j2.push_back(j2);
                for (int m2 = -j2; m2 <= j2; m2 += 2) {
                    h.orb_alpha.push_back(alpha);
                    h.orb_m2.push_back(m2);
                }
            }
    const int n = (int)h.nlj_N.size();
    h.tidx.assign((size_t)n * n * n, -1);
    for (int a = 0; a < n; a++)
        for (int b = 0; b < n; b++)
            for (int c = 0; c < n; c++)
                if (h.nlj_N[a] + h.nlj_N[b] + h.nlj_N[c] <= n3max) {
                    h.tidx[((size_t)a * n + b) * n + c] = (int32_t)(h.trip.size() / 3);
                    h.trip.push_back(a);
                    h.trip.push_back(b);
                    h.trip.push_back(c);
                }
    const int nt = (int)(h.trip.size() / 3);
    if (nt > 8192) {
        err = "more than 8192 orbital triples (lower n3max)";
        return CI_EUNSUPPORTED;
    }
    h.block_off.assign((size_t)nt * nt, -1);
    int64_t pos = 0;
    for (int t = 0; t < nt; t++) {
        const int* x = &h.trip[3 * t];
        const int jx[3] = {h.nlj_j2[x[0]], h.nlj_j2[x[1]], h.nlj_j2[x[2]]};
        const int px = (h.nlj_l[x[0]] + h.nlj_l[x[1]] + h.nlj_l[x[2]]) & 1;
        for (int u = 0; u < nt; u++) {
            const int* y = &h.trip[3 * u];
            const int jy[3] = {h.nlj_j2[y[0]], h.nlj_j2[y[1]], h.nlj_j2[y[2]]};
            if (((h.nlj_l[y[0]] + h.nlj_l[y[1]] + h.nlj_l[y[2]]) & 1) != px) continue;
            h.block_off[(size_t)t * nt + u] = pos;
            const int Jmax = std::min(jx[0] + jx[1] + jx[2], jy[0] + jy[1] + jy[2]);
            for (int J = 1; J <= Jmax; J += 2)
                for (int T = 1; T <= 3; T += 2)
                    pos += (int64_t)n_channels(jx[0], jx[1], jx[2], J, T) * n_channels(jy[0], jy[1], jy[2], J, T);
        }
    }
    h.n_coupled = pos;
    return CI_OK;
}

// Keys of the coupled elements in storage order: (t, t', 2J, 2T, 2J_ab,
// 2T_ab, 2J_de, 2T_de) per element.
void threebody_keys(const ThreeBodyHost& h, int32_t* keys)
{
    const int nt = (int)(h.trip.size() / 3);
    int64_t pos = 0;
    for (int t = 0; t < nt; t++)
        for (int u = 0; u < nt; u++) {
            if (h.block_off[(size_t)t * nt + u] < 0) continue;
            const int* x = &h.trip[3 * t];
            const int* y = &h.trip[3 * u];
            const int jx[3] = {h.nlj_j2[x[0]], h.nlj_j2[x[1]], h.nlj_j2[x[2]]};
            const int jy[3] = {h.nlj_j2[y[0]], h.nlj_j2[y[1]], h.nlj_j2[y[2]]};
            const int Jmax = std::min(jx[0] + jx[1] + jx[2], jy[0] + jy[1] + jy[2]);
            for (int J = 1; J <= Jmax; J += 2)
                for (int T = 1; T <= 3; T += 2) {
                    if (!n_channels(jx[0], jx[1], jx[2], J, T) || !n_channels(jy[0], jy[1], jy[2], J, T)) continue;
                    for (int jab = std::abs(jx[0] - jx[1]); jab <= jx[0] + jx[1]; jab += 2) {
                        if (!triangle2(jab, jx[2], J)) continue;
                        for (int tab = 0; tab <= 2; tab += 2) {
                            if (!triangle2(tab, 1, T)) continue;
                            for (int jde = std::abs(jy[0] - jy[1]); jde <= jy[0] + jy[1]; jde += 2) {
                                if (!triangle2(jde, jy[2], J)) continue;
                                for (int tde = 0; tde <= 2; tde += 2) {
                                    if (!triangle2(tde, 1, T)) continue;
                                    int32_t* k = keys + 8 * pos++;
                                    k[0] = t;
                                    k[1] = u;
                                    k[2] = J;
                                    k[3] = T;
                                    k[4] = jab;
                                    k[5] = tab;
                                    k[6] = jde;
                                    k[7] = tde;
                                }
                            }
                        }
                    }
                }
        }
}

// Device tables of the layout and the coefficient tables: built contiguously
// on the host and moved with one allocation and one copy (paper Sec. 3.3).
hipError_t threebody_upload(ThreeBodyHost& h)
{
    const int nj = h.n1max + 1;
    std::vector<int32_t> off1, off2;
    std::vector<float> cg1, cg2;
    build_cg_tables(nj, off1, cg1, off2, cg2);
    std::vector<char> mirror;
    auto put = [&](const void* src, size_t n) {
        const size_t o = mirror.size();
        mirror.resize(o + (n + 255) / 256 * 256, 0);
        std::memcpy(mirror.data() + o, src, n);
        return o;
    };
    std::vector<uint32_t> orb(h.orb_alpha.size());
    for (size_t q = 0; q < orb.size(); q++) {
        const int a = h.orb_alpha[q];
        orb[q] = (uint32_t)a | (uint32_t)h.nlj_j2[a] << 8 | (uint32_t)(h.orb_m2[q] + 64) << 16 |
                 (uint32_t)h.nlj_l[a] << 24;
    }
    const size_t o0 = put(orb.data(), orb.size() * 4);
    const size_t o4 = put(h.tidx.data(), h.tidx.size() * 4);
    const size_t o5 = put(h.block_off.data(), h.block_off.size() * 8);
    const size_t o6 = put(off1.data(), off1.size() * 4);
    const size_t o7 = put(off2.data(), off2.size() * 4);
    const size_t o8 = put(cg1.data(), cg1.size() * 4);
    const size_t o9 = put(cg2.data(), cg2.size() * 4);
    hipError_t e = hipMalloc(&h.arena, mirror.size());
    if (e != hipSuccess) return e;
    e = hipMemcpy(h.arena, mirror.data(), mirror.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    char* d = (char*)h.arena;
    h.dev.nsps = (int32_t)h.orb_alpha.size();
    h.dev.nlj = (int32_t)h.nlj_j2.size();
    h.dev.ntrip = (int32_t)(h.trip.size() / 3);
    h.dev.nj = nj;
    h.dev.orb = (const uint32_t*)(d + o0);
    h.dev.tidx = (const int32_t*)(d + o4);
    h.dev.block_off = (const int64_t*)(d + o5);
    h.dev.cg1_off = (const int32_t*)(d + o6);
    h.dev.cg2_off = (const int32_t*)(d + o7);
    h.dev.cg1 = (const float*)(d + o8);
    h.dev.cg2 = (const float*)(d + o9);
    return hipSuccess;
}

void threebody_release(ThreeBodyHost& h)
{
    if (h.arena) (void)hipFree(h.arena);
    h.arena = nullptr;
}

size_t decouple_work_bytes(int64_t n)
{
    if (n <= 0) return 0;
    return (size_t)2 * kCounters * 4 + (size_t)(n + 255) / 256 * 256 + (size_t)n * 4;
}

hipError_t launch_decouple(const ThreeBodyHost& h, const float* A, const int32_t* req, int64_t n, void* work,
                           float* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int32_t* order = nullptr;
    if (work) {
        uint32_t* counters = (uint32_t*)work;  // [2][kCostBins][kCostReplicas]: counts, then cursors
        uint8_t* bin = (uint8_t*)work + (size_t)2 * kCounters * 4;
        int32_t* ord = (int32_t*)(bin + (size_t)(n + 255) / 256 * 256);
        const unsigned blocks = (unsigned)((n + kOrderPerBlock - 1) / kOrderPerBlock);
        hipLaunchKernelGGL(order_clear, dim3(1), dim3(1024), 0, s, counters);
        hipLaunchKernelGGL(order_histogram, dim3(blocks), dim3(kOrderThreads), 0, s, h.dev, req, n, bin, counters);
        hipLaunchKernelGGL(order_starts, dim3(1), dim3(256), 0, s, counters);
        hipLaunchKernelGGL(order_scatter, dim3(blocks), dim3(kOrderThreads), 0, s, bin, n, counters + kCounters,
                           ord);
        order = ord;
    }
    hipLaunchKernelGGL(decouple_kernel, dim3((unsigned)((n + kDecoupleThreads - 1) / kDecoupleThreads)),
                       dim3(kDecoupleThreads), decouple_lds_bytes(h.dev.nj), s, h.dev, A, req, n, order, out);
    return hipGetLastError();
}

}  // namespace ci
