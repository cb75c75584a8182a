// Many-body matrix with a three-body term (paper Sec. 2: the elements are
// combinations of kinetic, two-body and three-body terms; Sec. 4.1: locate,
// then calculate and store, half of the symmetric matrix).
//
// Stored entries: every pair of basis states i <= j that differ in at most
// three nucleons, structural zeros included, columns ascending.  Values:
// one- and two-body part as for the two-body matrix (d <= 2), plus the
// three-body part by the Slater-Condon rules with particles p (in row i, not
// in column j), holes h (in j, not in i) and spectators (in both):
//   d = 0: sum over occupied a < b < c of V_{abc,abc}
//   d = 1: phase * sum over spectators k < l of V_{pkl,hkl}
//   d = 2: phase * sum over spectators k of V_{p1 p2 k, h1 h2 k}
//   d = 3: phase * V_{p1 p2 p3, h1 h2 h3}
// The phase removes the holes from the column state in ascending order and
// adds the particles in descending order.  The paper's three-body elements
// come from its decoupling (Sec. 3); here they are synthetic: the (x+1)-th
// output of the splitmix64 generator (Steele, Lea & Flood 2014) for the
// canonical pair of ascending triples, or the identity.
//
// Work: one wavefront per row.  The row walks the blocks at and after its
// own, 64 proton determinants of the block's proton key at a time.  A proton
// partner three nucleons away leaves only the row's own neutron determinant
// (one entry); two away, the one-neutron partners of the row's neutron
// determinant (its partner list); one or zero away, the wavefront scans the
// neutron key together.  An in-wave prefix sum over the 64 proton lanes
// places every entry, so columns come out ascending.  Count and fill run the
// same walk.
#include <hip/hip_runtime.h>

#include "ci_internal.h"

namespace ci {

namespace {

constexpr int kH3Waves = 4;
constexpr int kH3MaxA = 128;  // nucleons of a row kept in LDS

struct V3Param {
    int kind;  // 0 none, 1 synthetic, 2 identity
    uint64_t seed;
    double scale;
};

template <typename T>
using cptr3 = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr3<T> uni(const T* p)
{
    return (cptr3<T>)p;
}

typedef int i32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ BlockInfo load_block(const BlockInfo* blk, int b)
{
    const i32x4_t v = *uni((const i32x4_t*)(blk + b));
    BlockInfo r;
    r.kp = v.x;
    r.kn = v.y;
    r.row0 = v.z;
    r.nkn = v.w;
    return r;
}

__device__ __forceinline__ void wave_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive prefix sum over the 64 lanes (DPP row shifts, row broadcasts)
__device__ __forceinline__ int incl_scan64(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return v;
}

__device__ __forceinline__ int read_lane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// k-th output of splitmix64 started at `state`
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t state, uint64_t k)
{
    uint64_t z = state + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// V_{abc,def} for ascending triples of combined orbit indices
__device__ double v3_sorted(const V3Param& v, int a, int b, int c, int d, int e, int f)
{
    if (v.kind == 2) return (a == d && b == e && c == f) ? v.scale : 0.0;
    const uint64_t kb = ((uint64_t)a * 512 + (uint64_t)b) * 512 + (uint64_t)c;
    const uint64_t kk = ((uint64_t)d * 512 + (uint64_t)e) * 512 + (uint64_t)f;
    const uint64_t lo = kb < kk ? kb : kk, hi = kb < kk ? kk : kb;
    const uint64_t z = splitmix64_at(v.seed, ((lo << 27) | hi) + 1);
    return v.scale * (2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0);
}

// V_{abc,def} for triples in any order (distinct orbits): sorted with the
// sign of both sorting permutations
__device__ double v3_any(const V3Param& v, int a, int b, int c, int d, int e, int f)
{
    bool neg = false;
    if (a > b) { const int t = a; a = b; b = t; neg = !neg; }
    if (b > c) { const int t = b; b = c; c = t; neg = !neg; }
    if (a > b) { const int t = a; a = b; b = t; neg = !neg; }
    if (d > e) { const int t = d; d = e; e = t; neg = !neg; }
    if (e > f) { const int t = e; e = f; f = t; neg = !neg; }
    if (d > e) { const int t = d; d = e; e = t; neg = !neg; }
    const double x = v3_sorted(v, a, b, c, d, e, f);
    return neg ? -x : x;
}

// Two-body element V_{ab,cd} (combined indices, any order; distinct within a
// pair), 0 when a pair is outside the table.  tb points at this basis' slice.
__device__ double v2_any(const BasisDev& B, const float* tb, int a, int b, int c, int d)
{
    bool neg = false;
    if (a > b) { const int t = a; a = b; b = t; neg = !neg; }
    if (c > d) { const int t = c; c = d; d = t; neg = !neg; }
    const int n = B.nsps;
    const int cls = (a >= n) + (b >= n);
    if (cls != (c >= n) + (d >= n)) return 0.0;
    a -= a >= n ? n : 0;
    b -= b >= n ? n : 0;
    c -= c >= n ? n : 0;
    d -= d >= n ? n : 0;
    const uint64_t* P = B.pair + (size_t)cls * n * n;
    const uint64_t e1 = P[a * n + b], e2 = P[c * n + d];
    const uint32_t l1 = (uint32_t)e1, l2 = (uint32_t)e2;
    if (e1 == kNoPair64 || e2 == kNoPair64 || (l1 >> 16) != (l2 >> 16)) return 0.0;
    const bool first = (l1 & 0xffff) <= (l2 & 0xffff);
    const uint32_t pos = (first ? (uint32_t)(e1 >> 32) : (uint32_t)(e2 >> 32)) + (first ? (l2 & 0xffff) : (l1 & 0xffff));
    const double x = (double)tb[pos];
    return neg ? -x : x;
}

// oscillator kinetic element between species-local orbits p != h of one
// species: (hw/2) sqrt((n+1)(n+l+3/2)) for radial n, n+1 of the same (l, j, m)
__device__ double kinetic_pair(const BasisDev& B, int p, int h)
{
    const int qp = B.orb_qn[p], qh = B.orb_qn[h];
    if ((qp >> 8) != (qh >> 8)) return 0.0;
    const int np = qp & 255, nh = qh & 255, l = (qp >> 8) & 255;
    const int lo = np < nh ? np : nh, hi = np < nh ? nh : np;
    if (hi != lo + 1) return 0.0;
    return 0.5 * B.hw * sqrt((double)(lo + 1) * ((double)lo + l + 1.5));
}

// occupied orbits of the column state below combined orbit o
template <int W>
__device__ __forceinline__ int below(const uint64_t* yp, const uint64_t* yn, int n, int Z, int o)
{
    const bool prot = o < n;
    const int q = prot ? o : o - n;
    int c = prot ? 0 : Z;
#pragma unroll
    for (int w = 0; w < W; w++) {
        const uint64_t y = prot ? yp[w] : yn[w];
        if (w < (q >> 6)) c += __popcll(y);
        else if (w == (q >> 6)) c += __popcll(y & ((1ull << (q & 63)) - 1));
    }
    return c;
}

// the k-th of up to three orbits packed 10 bits each
__device__ __forceinline__ int unpack3(int v, int k) { return (v >> (10 * k)) & 1023; }

// <row|H|column> for states at most three nucleons apart: row words xp, xn,
// column words yp, yn, the row's occupied orbits occ[A] (combined, ascending).
template <int W>
__device__ double entry_value(const BasisDev& B, const float* tb, const V3Param& v3, const uint64_t* xp,
                              const uint64_t* xn, const uint64_t* yp, const uint64_t* yn, const int16_t* occ)
{
    const int n = B.nsps, A = B.Z + B.NN;
    // particles (row, not column) and holes (column, not row), ascending,
    // packed 10 bits each
    int P = 0, H = 0, d = 0, dh = 0;
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
        for (int w = 0; w < W; w++) {
            const uint64_t X = s ? xn[w] : xp[w], Y = s ? yn[w] : yp[w];
            uint64_t pm = X & ~Y, hm = Y & ~X;
            while (pm) {
                P |= (s * n + w * 64 + __builtin_ctzll(pm)) << (10 * d++);
                pm &= pm - 1;
            }
            while (hm) {
                H |= (s * n + w * 64 + __builtin_ctzll(hm)) << (10 * dh++);
                hm &= hm - 1;
            }
        }
    double v = 0.0;
    if (d == 0) {
        for (int a = 0; a < A; a++) {
            const int oa = occ[a];
            v += (B.orb_n[oa < n ? oa : oa - n] + 1.5) * B.hw * (B.kinetic ? 0.5 : 1.0);
            for (int b = a + 1; b < A; b++) {
                v += v2_any(B, tb, oa, occ[b], oa, occ[b]);
                if (v3.kind)
                    for (int c = b + 1; c < A; c++) v += v3_sorted(v3, oa, occ[b], occ[c], oa, occ[b], occ[c]);
            }
        }
        return v;
    }
    const int p0 = unpack3(P, 0), p1 = unpack3(P, 1), p2 = unpack3(P, 2);
    const int h0 = unpack3(H, 0), h1 = unpack3(H, 1), h2 = unpack3(H, 2);
    int e = -d * (d - 1) / 2;
    for (int k = 0; k < d; k++) {
        const int pk = unpack3(P, k);
        e += below<W>(yp, yn, n, B.Z, unpack3(H, k)) + below<W>(yp, yn, n, B.Z, pk);
        e -= (h0 < pk) + (d > 1 && h1 < pk) + (d > 2 && h2 < pk);
    }
    auto spectator = [&](int o) { return o != p0 && (d < 2 || o != p1) && (d < 3 || o != p2); };
    if (d == 1) {
        for (int a = 0; a < A; a++) {
            const int k = occ[a];
            if (!spectator(k)) continue;
            v += v2_any(B, tb, p0, k, h0, k);
            if (v3.kind)
                for (int b = a + 1; b < A; b++) {
                    const int l = occ[b];
                    if (spectator(l)) v += v3_any(v3, p0, k, l, h0, k, l);
                }
        }
        if (B.kinetic) v += kinetic_pair(B, p0 < n ? p0 : p0 - n, h0 < n ? h0 : h0 - n);
    } else if (d == 2) {
        v = v2_any(B, tb, p0, p1, h0, h1);
        if (v3.kind)
            for (int a = 0; a < A; a++) {
                const int k = occ[a];
                if (spectator(k)) v += v3_any(v3, p0, p1, k, h0, h1, k);
            }
    } else if (v3.kind) {
        v = v3_sorted(v3, p0, p1, p2, h0, h1, h2);
    }
    return (e & 1) ? -v : v;
}

template <int W>
__device__ __forceinline__ int dist(const uint64_t* x, const uint64_t* y)
{
    int c = 0;
#pragma unroll
    for (int w = 0; w < W; w++) c += __popcll(x[w] ^ y[w]);
    return c >> 1;
}

// The move of one species between row words x and column words y:
// particles (in x, not y) and holes (in y, not x), ascending, as combined
// indices (species-local + base) packed 10 bits each, and the species' part
// of the phase, sum of below_y over holes and particles minus the
// (hole < particle) pairs.  Every proton orbit precedes every neutron orbit,
// so the phase of the whole move is e_p + e_n - dp*dn - d(d-1)/2 (mod 2).
struct Move {
    int P, H, e;
};

template <int W>
__device__ __forceinline__ Move species_move(const uint64_t* x, const uint64_t* y, int base)
{
    Move m{0, 0, 0};
    int np = 0, nh = 0, run = 0;  // run: column orbits of the words before w
#pragma unroll
    for (int w = 0; w < W; w++) {
        uint64_t pm = x[w] & ~y[w], hm = y[w] & ~x[w];
        while (pm) {
            const int b = __builtin_ctzll(pm);
            m.e += run + __popcll(y[w] & ((1ull << b) - 1));
            m.P |= (base + w * 64 + b) << (10 * np++);
            pm &= pm - 1;
        }
        while (hm) {
            const int b = __builtin_ctzll(hm);
            m.e += run + __popcll(y[w] & ((1ull << b) - 1));
            m.H |= (base + w * 64 + b) << (10 * nh++);
            hm &= hm - 1;
        }
        run += __popcll(y[w]);
    }
    // (hole < particle) pairs inside the species
    for (int k = 0; k < np; k++)
        for (int q = 0; q < nh; q++) m.e -= unpack3(m.H, q) < unpack3(m.P, k);
    return m;
}

// Value of an entry three nucleons apart from the moves of both species
// (dp + dn = 3): the phase times V_{particles, holes}.
__device__ __forceinline__ double value3(const V3Param& v3, const Move& mp, int dp, const Move& mn)
{
    if (!v3.kind) return 0.0;
    const int Pc = mp.P | (mn.P << (10 * dp)), Hc = mp.H | (mn.H << (10 * dp));
    const double v = v3_sorted(v3, unpack3(Pc, 0), unpack3(Pc, 1), unpack3(Pc, 2), unpack3(Hc, 0), unpack3(Hc, 1),
                               unpack3(Hc, 2));
    const int e = mp.e + mn.e - dp * (3 - dp) - 3;
    return (e & 1) ? -v : v;
}

// Partner index of the three-body walk, per species: for every determinant x
// and every key, the determinants y of that key with d(x, y) <= 2, ascending
// (the two-body path's lists hold d <= 1 in every key but d = 2 only in keys
// of x's own 2M and parity; a proton one nucleon away moves the neutron key).  Records use the two-body partner layout (local
// index, h1, p1, h2, p2, d); the sign bit holds the parity of the move's
// species phase part (sum of below_y over holes and particles minus the
// hole < particle pairs), which for d <= 1 is the two-body record's sign.
struct H3Index {
    const int32_t* seg;  // [nsd][nk + 1] first record of each key in x's list
    const int64_t* ptr;  // [nsd + 1] start of x's list
    const uint64_t* rec;
};

struct H3Indexes {
    H3Index n, p;  // neutrons, protons
};

template <bool kFill, int W>
__global__ void __launch_bounds__(64 * kH3Waves) h3_index(const BasisDev* __restrict__ Bp, int species,
                                                          int32_t* __restrict__ seg, int64_t* __restrict__ ptr,
                                                          uint64_t* __restrict__ rec)
{
    const BasisDev B = *Bp;
    const SpeciesDev& S = B.sp[species];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t x = (int64_t)blockIdx.x * kH3Waves + wave;
    if (!kFill && x == 0 && lane == 0) ptr[0] = 0;
    if (x >= S.nsd) return;
    uint64_t xw[W];
#pragma unroll
    for (int w = 0; w < W; w++) xw[w] = uni(S.sd)[x * W + w];
    const int64_t base = kFill ? uni(ptr)[x] : 0;
    int run = 0;
    for (int k = 0; k < S.nk; k++) {
        if (!kFill && lane == 0) seg[x * (S.nk + 1) + k] = run;
        const int y0 = uni(S.key_off)[k], y1 = uni(S.key_off)[k + 1];
        for (int c = y0; c < y1; c += 64) {
            const int y = c + lane;
            uint64_t yw[W];
#pragma unroll
            for (int w = 0; w < W; w++) yw[w] = y < y1 ? S.sd[(int64_t)y * W + w] : 0ull;
            const int d = dist<W>(xw, yw);
            const bool ok = y < y1 && d <= 2;
            const uint64_t m = __ballot(ok);
            if (kFill && ok) {
                const Move mv = species_move<W>(xw, yw, 0);
                const int p1 = unpack3(mv.P, 0), p2 = unpack3(mv.P, 1), h1 = unpack3(mv.H, 0), h2 = unpack3(mv.H, 1);
                rec[base + run + __popcll(m & ((1ull << lane) - 1))] =
                    make_rec((uint32_t)(y - y0), d, d >= 1 ? h1 : 0, d >= 1 ? p1 : 0, d == 2 ? h2 : 0,
                             d == 2 ? p2 : 0, (mv.e & 1) != 0);
            }
            run += __popcll(m);
        }
    }
    if (!kFill && lane == 0) {
        seg[x * (S.nk + 1) + S.nk] = run;
        ptr[x + 1] = run;
    }
}

// The neutron move of a partner record (orbits species-local + base): the
// particles p1 (< p2), holes h1 (< h2), and the phase part from the sign bit.
__device__ __forceinline__ Move rec_move(uint64_t rc, int base)
{
    const int d = (int)((rc >> 57) & 3);
    Move m{0, 0, (int)((rc >> 56) & 1)};
    if (d >= 1) {
        m.P = base + (int)((rc >> 32) & 255);
        m.H = base + (int)((rc >> 24) & 255);
    }
    if (d == 2) {
        m.P |= (base + (int)((rc >> 48) & 255)) << 10;
        m.H |= (base + (int)((rc >> 40) & 255)) << 10;
    }
    return m;
}

// Entries at most two nucleons apart found by the wavefront's joint neutron
// scans cost 4 to 30 three-body terms, the others (three apart) one; mixed in
// one wavefront every lane would wait for the dearest.  The scan computes the
// three-apart values at once and queues the others by class (two apart; one
// or zero apart), 64 per batch, one entry per lane.
struct H3Queue {
    int32_t pos[64];  // offset from the row's first entry
    int32_t pg[64];   // proton determinant (global index)
    int32_t ng[64];   // neutron determinant (global index)
};

template <bool kFill, int W>
__global__ void __launch_bounds__(64 * kH3Waves) h3_rows(const BasisDev* __restrict__ Bp, H3Indexes X,
                                                         const float* __restrict__ tbme, V3Param v3,
                                                         int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                         float* __restrict__ val, int full)
{
    __shared__ int16_t occ_s[kH3Waves][kH3MaxA];
    __shared__ H3Queue queue_s[kH3Waves][2];
    __shared__ uint8_t lanes_s[kH3Waves][64];
    const BasisDev B = *Bp;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * kH3Waves + wave;
    if (!kFill && i == 0 && lane == 0) row_ptr[B.row0] = 0;
    if (i >= B.dim) return;
    const SpeciesDev& SP = B.sp[0];
    const SpeciesDev& SN = B.sp[1];
    // block of the row
    int lo = 0, hi = B.nblk;  // blk_off[lo] <= i < blk_off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (uni(B.blk_off)[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int b = lo;
    const BlockInfo bi = load_block(B.blk, b);
    const int ip = (int)((i - bi.row0) / bi.nkn), in = (int)((i - bi.row0) % bi.nkn);
    const int pg = uni(SP.key_off)[bi.kp] + ip, ng = uni(SN.key_off)[bi.kn] + in;
    uint64_t xp[W], xn[W];
#pragma unroll
    for (int w = 0; w < W; w++) {
        xp[w] = uni(SP.sd)[(int64_t)pg * W + w];
        xn[w] = uni(SN.sd)[(int64_t)ng * W + w];
    }
    int16_t* occ = occ_s[wave];
    if (kFill) {
        if (lane == 0) {
            int k = 0;
#pragma unroll
            for (int s = 0; s < 2; s++)
#pragma unroll
                for (int w = 0; w < W; w++) {
                    uint64_t m = s ? xn[w] : xp[w];
                    while (m) {
                        occ[k++] = (int16_t)(s * B.nsps + w * 64 + __builtin_ctzll(m));
                        m &= m - 1;
                    }
                }
        }
        wave_fence();
    }
    const float* tb = tbme ? tbme + B.tbme0 : nullptr;
    const int32_t* seg = SN.seg1 + (int64_t)ng * (SN.nk + 1);
    const uint64_t* rec1 = SN.l1 + uni(SN.l1_ptr)[ng];
    const int32_t* seg2 = X.n.seg + (int64_t)ng * (SN.nk + 1);
    const uint64_t* rec2 = X.n.rec + uni(X.n.ptr)[ng];
    const int32_t* segP = X.p.seg + (int64_t)pg * (SP.nk + 1);
    const uint64_t* recP = X.p.rec + uni(X.p.ptr)[pg];
    int64_t out = kFill ? uni(row_ptr)[B.row0 + i] : 0;
    const int64_t row_start = out;
    H3Queue* Q = queue_s[wave];
    int nq[2] = {0, 0};
    auto flush = [&](int k) {
        wave_fence();
        if (lane < nq[k]) {
            const int64_t gp = Q[k].pg[lane], gn = Q[k].ng[lane];
            uint64_t yp2[W], yn2[W];
#pragma unroll
            for (int w = 0; w < W; w++) {
                yp2[w] = SP.sd[gp * W + w];
                yn2[w] = SN.sd[gn * W + w];
            }
            val[row_start + Q[k].pos[lane]] = (float)entry_value<W>(B, tb, v3, xp, xn, yp2, yn2, occ);
        }
        wave_fence();
        nq[k] = 0;
    };
    // full: every column of the row (both triangles); else j >= i
    for (int b2 = full ? 0 : b; b2 < B.nblk; b2++) {
        const BlockInfo bj = load_block(B.blk, b2);
        const int kp0 = uni(SP.key_off)[bj.kp], nKp = uni(SP.key_off)[bj.kp + 1] - kp0;
        const int kn0 = uni(SN.key_off)[bj.kn], nKn = bj.nkn;
        const bool same_n = bj.kn == bi.kn;
        const int s0 = uni(seg)[bj.kn], n_le1 = uni(seg)[bj.kn + 1] - s0;  // neutrons of the key at most one away
        const int r0 = uni(seg2)[bj.kn], r1 = uni(seg2)[bj.kn + 1];  // ... at most two away
        // one step: 64 proton determinants of the block's proton key (pl their
        // local index, dp their distance, mp their move when filling)
        auto step = [&](int pl, int dp, const Move& mp) {
            int cnt = dp == 3 ? (same_n ? 1 : 0) : dp == 2 ? n_le1 : dp == 1 ? r1 - r0 : 0;
            // the row's own proton determinant (zero away): the wavefront scans the neutron key
            uint64_t coop = __ballot(dp == 0);
            while (coop) {
                const int L = __builtin_ctzll(coop);
                coop &= coop - 1;
                const int excl = read_lane(incl_scan64(cnt) - cnt, L);
                const int pL = read_lane(pl, L);
                int found = 0;
                for (int nc = (!full && b2 == b && pL == ip ? in : 0); nc < nKn; nc += 64) {
                    const int nl = nc + lane;
                    uint64_t yn[W];
#pragma unroll
                    for (int w = 0; w < W; w++) yn[w] = nl < nKn ? SN.sd[(int64_t)(kn0 + nl) * W + w] : 0ull;
                    const int dn = dist<W>(xn, yn);
                    const bool ok = nl < nKn && dn <= 3;
                    const uint64_t m = __ballot(ok);
                    if (kFill) {
                        const uint64_t below_lane = (1ull << lane) - 1;
                        const int cls = !ok ? -1 : dn == 3 ? 2 : dn == 2 ? 0 : 1;
                        const uint64_t mq[2] = {__ballot(cls == 0), __ballot(cls == 1)};
                        for (int k = 0; k < 2; k++)
                            if (nq[k] + __popcll(mq[k]) > 64) flush(k);
                        const int64_t pos = out + excl + found + __popcll(m & below_lane);
                        if (ok) col[pos] = bj.row0 + pL * nKn + nl;
                        if (cls == 2) val[pos] = (float)value3(v3, Move{0, 0, 0}, 0, species_move<W>(xn, yn, B.nsps));
                        if (cls == 0 || cls == 1) {
                            const int k = nq[cls] + __popcll(mq[cls] & below_lane);
                            Q[cls].pos[k] = (int32_t)(pos - row_start);
                            Q[cls].pg[k] = kp0 + pL;
                            Q[cls].ng[k] = kn0 + nl;
                        }
                        nq[0] += __popcll(mq[0]);
                        nq[1] += __popcll(mq[1]);
                    }
                    found += __popcll(m);
                }
                if (lane == L) cnt = found;
            }
            const int incl = incl_scan64(cnt), excl = incl - cnt;
            if (kFill) {
                if (cnt > 0 && dp == 3) {
                    col[out + excl] = bj.row0 + pl * nKn + in;
                    val[out + excl] = (float)value3(v3, mp, 3, Move{0, 0, 0});
                }
                // (proton, neutron record) pairs, 64 per step: one proton away
                // with the neutrons at most two away, two away with those at
                // most one away (the two-body path's list)
                uint8_t* lanes = lanes_s[wave];
                const uint64_t below_lane = (1ull << lane) - 1;
                for (int cp = 1; cp <= 2; cp++) {
                    const uint64_t mk = __ballot(dp == cp);
                    const int nr = cp == 1 ? r1 - r0 : n_le1;
                    const int total = __popcll(mk) * nr;
                    if (total == 0) continue;
                    if (dp == cp) lanes[__popcll(mk & below_lane)] = (uint8_t)lane;
                    wave_fence();
                    for (int t0 = 0; t0 < total; t0 += 64) {
                        const int t = t0 + lane;
                        const bool act = t < total;
                        const int j = act ? t / nr : 0, r = act ? t - j * nr : 0;
                        const int L = lanes[j];
                        const int plL = __builtin_amdgcn_ds_bpermute(L << 2, pl);
                        const int exL = __builtin_amdgcn_ds_bpermute(L << 2, excl);
                        const Move mpL{__builtin_amdgcn_ds_bpermute(L << 2, mp.P),
                                       __builtin_amdgcn_ds_bpermute(L << 2, mp.H),
                                       __builtin_amdgcn_ds_bpermute(L << 2, mp.e)};
                        // the neutron record carries its move: no determinant words needed
                        const uint64_t rc = !act ? 0ull : cp == 1 ? rec2[r0 + r] : rec1[s0 + r];
                        const int nl = (int)(rc & kRecLocalMask), dn = (int)((rc >> 57) & 3);
                        const int cls = !act ? -1 : cp + dn == 3 ? 2 : cp + dn == 2 ? 0 : 1;
                        const uint64_t mq[2] = {__ballot(cls == 0), __ballot(cls == 1)};
                        for (int k = 0; k < 2; k++)
                            if (nq[k] + __popcll(mq[k]) > 64) flush(k);
                        const int64_t pos = out + exL + r;
                        if (act) col[pos] = bj.row0 + plL * nKn + nl;
                        if (cls == 2) val[pos] = (float)value3(v3, mpL, cp, rec_move(rc, B.nsps));
                        if (cls == 0 || cls == 1) {
                            const int k = nq[cls] + __popcll(mq[cls] & below_lane);
                            Q[cls].pos[k] = (int32_t)(pos - row_start);
                            Q[cls].pg[k] = kp0 + plL;
                            Q[cls].ng[k] = kn0 + nl;
                        }
                        nq[0] += __popcll(mq[0]);
                        nq[1] += __popcll(mq[1]);
                    }
                    wave_fence();
                }
            }
            out += read_lane(incl, 63);
        };
        if (same_n) {
            // the block holds the row's neutron key: every proton determinant
            // up to three away contributes; scan the proton key
            for (int c = (!full && b2 == b ? ip : 0); c < nKp; c += 64) {
                const int pl = c + lane;
                uint64_t yp[W];
                int dp = 4;
#pragma unroll
                for (int w = 0; w < W; w++) yp[w] = pl < nKp ? SP.sd[(int64_t)(kp0 + pl) * W + w] : 0ull;
                if (pl < nKp) dp = dist<W>(xp, yp);
                Move mp{0, 0, 0};
                if (kFill && dp <= 3) mp = species_move<W>(xp, yp, 0);
                step(pl, dp, mp);
            }
        } else {
            // only proton determinants at most two away contribute: walk the
            // row's proton partner index in this key (moves in the records)
            const int q0 = uni(segP)[bj.kp], q1 = uni(segP)[bj.kp + 1];
            for (int c = q0; c < q1; c += 64) {
                const int r = c + lane;
                const uint64_t rc = r < q1 ? recP[r] : 0ull;
                step((int)(rc & kRecLocalMask), r < q1 ? (int)((rc >> 57) & 3) : 4, rec_move(rc, 0));
            }
        }
    }
    if (kFill) {
        flush(0);
        flush(1);
    }
    if (!kFill && lane == 0) row_ptr[B.row0 + i + 1] = out;
}

}  // namespace

template <int W>
static void launch_one(bool fill, unsigned grid, const BasisDev* B, const H3Indexes& X, const float* tbme,
                       const V3Param& v3, int64_t* row_ptr, int32_t* col, float* val, int full, hipStream_t s)
{
    if (fill)
        hipLaunchKernelGGL((h3_rows<true, W>), dim3(grid), dim3(64 * kH3Waves), 0, s, B, X, tbme, v3, row_ptr, col,
                           val, full);
    else
        hipLaunchKernelGGL((h3_rows<false, W>), dim3(grid), dim3(64 * kH3Waves), 0, s, B, X, tbme, v3, row_ptr, col,
                           val, full);
}

template <int W>
static void launch_index(bool fill, unsigned grid, const BasisDev* B, int species, int32_t* seg, int64_t* ptr,
                         uint64_t* rec, hipStream_t s)
{
    if (fill)
        hipLaunchKernelGGL((h3_index<true, W>), dim3(grid), dim3(64 * kH3Waves), 0, s, B, species, seg, ptr, rec);
    else
        hipLaunchKernelGGL((h3_index<false, W>), dim3(grid), dim3(64 * kH3Waves), 0, s, B, species, seg, ptr, rec);
}

// Partner index of one species of one basis (nsd determinants, W words):
// pass 1 writes seg and the list lengths into ptr[1..nsd] (ptr[0] = 0; the
// caller scans ptr), pass 2 the records.
hipError_t launch_h3_index(bool fill, const BasisDev* B, int species, int64_t nsd, int W, int32_t* seg, int64_t* ptr,
                           uint64_t* rec, hipStream_t s)
{
    const unsigned grid = (unsigned)((nsd + kH3Waves - 1) / kH3Waves);
    if (grid == 0) return hipSuccess;
    switch (W) {
    case 1: launch_index<1>(fill, grid, B, species, seg, ptr, rec, s); break;
    case 2: launch_index<2>(fill, grid, B, species, seg, ptr, rec, s); break;
    case 3: launch_index<3>(fill, grid, B, species, seg, ptr, rec, s); break;
    default: launch_index<4>(fill, grid, B, species, seg, ptr, rec, s); break;
    }
    return hipGetLastError();
}

// One launch per basis of the handle: count (row_ptr[R_b + 1 + i] = entries
// of row i, row_ptr[R_b] = 0) or fill (entries at row_ptr[R_b + i]); full:
// every column of a row, else the upper triangle.
// words[p]: 64-bit words per species bitstring of basis p (1..4); index[6p..]:
// its neutron, then proton, partner index (seg, ptr, rec).
hipError_t launch_h3_rows(const BasisDev* bases, const int64_t* dims, const int* words, const void* const* index,
                          int nb, const float* tbme, int v3_kind, uint64_t v3_seed, double v3_scale, int64_t* row_ptr,
                          int32_t* col, float* val, bool fill, int full, hipStream_t s)
{
    const V3Param v3{v3_kind, v3_seed, v3_scale};
    for (int p = 0; p < nb; p++) {
        // an empty basis still owns its first row_ptr slot (written by the count)
        const unsigned grid = (unsigned)((dims[p] + kH3Waves - 1) / kH3Waves);
        if (grid == 0 && fill) continue;
        const unsigned g = grid > 0 ? grid : 1;
        const H3Indexes X{{(const int32_t*)index[6 * p], (const int64_t*)index[6 * p + 1], (const uint64_t*)index[6 * p + 2]},
                          {(const int32_t*)index[6 * p + 3], (const int64_t*)index[6 * p + 4],
                           (const uint64_t*)index[6 * p + 5]}};
        switch (words[p]) {
        case 1: launch_one<1>(fill, g, bases + p, X, tbme, v3, row_ptr, col, val, full, s); break;
        case 2: launch_one<2>(fill, g, bases + p, X, tbme, v3, row_ptr, col, val, full, s); break;
        case 3: launch_one<3>(fill, g, bases + p, X, tbme, v3, row_ptr, col, val, full, s); break;
        default: launch_one<4>(fill, g, bases + p, X, tbme, v3, row_ptr, col, val, full, s); break;
        }
    }
    return hipGetLastError();
}

}  // namespace ci
