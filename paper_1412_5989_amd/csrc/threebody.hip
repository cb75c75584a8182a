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
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "ci_internal.h"

namespace ci {

namespace {

__host__ __device__ __forceinline__ bool triangle2(int a2, int b2, int c2)
{
    const int d = a2 > b2 ? a2 - b2 : b2 - a2;
    return d <= c2 && c2 <= a2 + b2 && ((a2 + b2 + c2) & 1) == 0;
}

// <j1 m1 j2 m2 | J M> (all arguments doubled) by the Racah formula; fact[n] = n!
__host__ __device__ double cg2(const double* fact, int j1, int m1, int j2, int m2, int J, int M)
{
    if (m1 + m2 != M) return 0.0;
    if (m1 > j1 || -m1 > j1 || m2 > j2 || -m2 > j2 || M > J || -M > J) return 0.0;
    if (((j1 + m1) & 1) || ((j2 + m2) & 1) || ((J + M) & 1) || !triangle2(j1, j2, J)) return 0.0;
    const int a = (j1 + j2 - J) / 2, b = (j1 - j2 + J) / 2, c = (-j1 + j2 + J) / 2, d = (j1 + j2 + J) / 2 + 1;
    const double pre = sqrt((double)(J + 1) * fact[a] * fact[b] * fact[c] / fact[d] * fact[(J + M) / 2] *
                            fact[(J - M) / 2] * fact[(j1 - m1) / 2] * fact[(j1 + m1) / 2] * fact[(j2 - m2) / 2] *
                            fact[(j2 + m2) / 2]);
    const int e1 = (j1 - m1) / 2, e2 = (j2 + m2) / 2, e3 = (J - j2 + m1) / 2, e4 = (J - j1 - m2) / 2;
    int kmin = 0;
    if (-e3 > kmin) kmin = -e3;
    if (-e4 > kmin) kmin = -e4;
    int kmax = a;
    if (e1 < kmax) kmax = e1;
    if (e2 < kmax) kmax = e2;
    double s = 0.0;
    for (int k = kmin; k <= kmax; k++) {
        const double t = 1.0 / (fact[k] * fact[a - k] * fact[e1 - k] * fact[e2 - k] * fact[e3 + k] * fact[e4 + k]);
        s += (k & 1) ? -t : t;
    }
    return pre * s;
}

// number of channels (J_ab, T_ab) of a triple with orbit spins ja, jb, jc
// (doubled) coupled to (J, T) (doubled)
__host__ __device__ __forceinline__ int n_channels(int ja, int jb, int jc, int J, int T)
{
    int n = 0;
    const int lo = ja > jb ? ja - jb : jb - ja;
    for (int jab = lo; jab <= ja + jb; jab += 2)
        if (triangle2(jab, jc, J))
            for (int tab = 0; tab <= 2; tab += 2)
                if (triangle2(tab, 1, T)) n++;
    return n;
}

constexpr int kFact = 96;  // n! up to 95!, enough for n1max <= 12

}  // namespace

namespace {

__global__ void __launch_bounds__(256) decouple_kernel(ThreeBodyDev T, const float* __restrict__ A,
                                                       const int32_t* __restrict__ req, int64_t n,
                                                       float* __restrict__ out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int o[6];
    bool ok = true;
    for (int k = 0; k < 6; k++) {
        o[k] = req[r * 6 + k];
        ok = ok && o[k] >= 0 && o[k] < 2 * T.nsps;
    }
    double sum = 0.0;
    if (ok) {
        int al[6], m[6], tz[6], j[6];
        for (int k = 0; k < 6; k++) {
            const int s = o[k] >= T.nsps, q = o[k] - s * T.nsps;
            al[k] = T.orb_alpha[q];
            m[k] = T.orb_m2[q];
            tz[k] = s ? -1 : 1;
            j[k] = T.nlj_j2[al[k]];
        }
        const int M = m[0] + m[1] + m[2], MT = tz[0] + tz[1] + tz[2];
        const int parb = (T.nlj_l[al[0]] + T.nlj_l[al[1]] + T.nlj_l[al[2]]) & 1;
        const int park = (T.nlj_l[al[3]] + T.nlj_l[al[4]] + T.nlj_l[al[5]]) & 1;
        const int n2 = T.nlj * T.nlj;
        const int tb = T.tidx[al[0] * n2 + al[1] * T.nlj + al[2]];
        const int tk = T.tidx[al[3] * n2 + al[4] * T.nlj + al[5]];
        if (M == m[3] + m[4] + m[5] && MT == tz[3] + tz[4] + tz[5] && parb == park && tb >= 0 && tk >= 0) {
            int64_t pos = T.block_off[(int64_t)tb * T.ntrip + tk];
            const int Jmax = min(j[0] + j[1] + j[2], j[3] + j[4] + j[5]);
            const int Mab = m[0] + m[1], Mde = m[3] + m[4], MTab = tz[0] + tz[1], MTde = tz[3] + tz[4];
            for (int J = 1; J <= Jmax && pos >= 0; J += 2)
                for (int TT = 1; TT <= 3; TT += 2) {
                    const int nb = n_channels(j[0], j[1], j[2], J, TT), nk = n_channels(j[3], j[4], j[5], J, TT);
                    if (nb == 0 || nk == 0) continue;
                    if (M <= J && -M <= J && MT <= TT && -MT <= TT) {
                        // bra channels in storage order: J_ab ascending, then T_ab
                        int ib = 0;
                        const int lob = abs(j[0] - j[1]);
                        for (int jab = lob; jab <= j[0] + j[1]; jab += 2) {
                            if (!triangle2(jab, j[2], J)) continue;
                            const double cj = cg2(T.fact, j[0], m[0], j[1], m[1], jab, Mab) *
                                              cg2(T.fact, jab, Mab, j[2], m[2], J, M);
                            for (int tab = 0; tab <= 2; tab += 2) {
                                if (!triangle2(tab, 1, TT)) continue;
                                const double cb = cj * cg2(T.fact, 1, tz[0], 1, tz[1], tab, MTab) *
                                                  cg2(T.fact, tab, MTab, 1, tz[2], TT, MT);
                                if (cb != 0.0) {
                                    int ik = 0;
                                    const int lok = abs(j[3] - j[4]);
                                    for (int jde = lok; jde <= j[3] + j[4]; jde += 2) {
                                        if (!triangle2(jde, j[5], J)) continue;
                                        const double ck = cg2(T.fact, j[3], m[3], j[4], m[4], jde, Mde) *
                                                          cg2(T.fact, jde, Mde, j[5], m[5], J, M);
                                        for (int tde = 0; tde <= 2; tde += 2) {
                                            if (!triangle2(tde, 1, TT)) continue;
                                            const double c = ck * cg2(T.fact, 1, tz[3], 1, tz[4], tde, MTde) *
                                                             cg2(T.fact, tde, MTde, 1, tz[5], TT, MT);
                                            if (c != 0.0) sum += cb * c * (double)A[pos + (int64_t)ib * nk + ik];
                                            ik++;
                                        }
                                    }
                                }
                                ib++;
                            }
                        }
                    }
                    pos += (int64_t)nb * nk;
                }
        }
    }
    out[r] = (float)sum;
}

}  // namespace

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

// Device tables of the layout: one allocation, one copy.
hipError_t threebody_upload(ThreeBodyHost& h)
{
    std::vector<double> fact(kFact, 1.0);
    for (int k = 1; k < kFact; k++) fact[k] = fact[k - 1] * k;
    auto bytes = [](size_t n, size_t s) { return (n * s + 255) / 256 * 256; };
    const size_t b0 = bytes(h.orb_alpha.size(), 4), b1 = bytes(h.orb_m2.size(), 4), b2 = bytes(h.nlj_j2.size(), 4),
                 b3 = bytes(h.nlj_l.size(), 4), b4 = bytes(h.tidx.size(), 4), b5 = bytes(h.trip.size(), 4),
                 b6 = bytes(h.block_off.size(), 8), b7 = bytes(fact.size(), 8);
    const size_t total = b0 + b1 + b2 + b3 + b4 + b5 + b6 + b7;
    std::vector<char> mirror(total, 0);
    size_t off = 0;
    auto put = [&](const void* src, size_t n, size_t b) {
        std::memcpy(mirror.data() + off, src, n);
        const size_t o = off;
        off += b;
        return o;
    };
    const size_t o0 = put(h.orb_alpha.data(), h.orb_alpha.size() * 4, b0);
    const size_t o1 = put(h.orb_m2.data(), h.orb_m2.size() * 4, b1);
    const size_t o2 = put(h.nlj_j2.data(), h.nlj_j2.size() * 4, b2);
    const size_t o3 = put(h.nlj_l.data(), h.nlj_l.size() * 4, b3);
    const size_t o4 = put(h.tidx.data(), h.tidx.size() * 4, b4);
    const size_t o5 = put(h.trip.data(), h.trip.size() * 4, b5);
    const size_t o6 = put(h.block_off.data(), h.block_off.size() * 8, b6);
    const size_t o7 = put(fact.data(), fact.size() * 8, b7);
    hipError_t e = hipMalloc(&h.arena, total);
    if (e != hipSuccess) return e;
    e = hipMemcpy(h.arena, mirror.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    char* d = (char*)h.arena;
    h.dev.nsps = (int32_t)h.orb_alpha.size();
    h.dev.nlj = (int32_t)h.nlj_j2.size();
    h.dev.ntrip = (int32_t)(h.trip.size() / 3);
    h.dev.orb_alpha = (const int32_t*)(d + o0);
    h.dev.orb_m2 = (const int32_t*)(d + o1);
    h.dev.nlj_j2 = (const int32_t*)(d + o2);
    h.dev.nlj_l = (const int32_t*)(d + o3);
    h.dev.tidx = (const int32_t*)(d + o4);
    h.dev.trip = (const int32_t*)(d + o5);
    h.dev.block_off = (const int64_t*)(d + o6);
    h.dev.fact = (const double*)(d + o7);
    return hipSuccess;
}

void threebody_release(ThreeBodyHost& h)
{
    if (h.arena) hipFree(h.arena);
    h.arena = nullptr;
}

hipError_t launch_decouple(const ThreeBodyHost& h, const float* A, const int32_t* req, int64_t n, float* out,
                           hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL(decouple_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h.dev, A, req, n,
                           out);
    return hipGetLastError();
}

}  // namespace ci
