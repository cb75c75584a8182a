// HIP kernels of libci for CDNA4 (gfx950): count, scan, fill and adjoint of
// the upper-triangle M-scheme Hamiltonian with a two-body interaction.
//
// Work unit: one wavefront per row i = (P, N) (proton determinant P, neutron
// determinant N).  Every stored column of row i is (P', N') with P' a
// proton partner of P (one- or two-proton move, or P itself) and N' a
// neutron partner of N.  Column order is block (Kp', Kn') ascending, then P',
// then N'; the partner lists are stored in that order (paper Sec. 4.1: for
// sparse chunks, iterate over the quantum-number combinations that can give a
// nonzero instead of testing every element).
//
// The row is produced by a two-level load-balanced expansion:
//   1. lanes take 64 target blocks at a time and count the proton partners
//      of P in each (a wave scan gives each block's first "segment");
//   2. lanes take 64 segments (target block, P') at a time and compute each
//      segment's number of entries from the neutron partner lists of N
//      (a wave scan gives each segment's first output position);
//   3. lanes take 64 consecutive entries at a time, find their segment by a
//      binary search in LDS, and write col/val: consecutive lanes write
//      consecutive addresses.
// Entries that differ in two nucleons are one signed two-body element and are
// finished in step 3.  The diagonal and one-nucleon differences are sums of
// many elements; they are queued in LDS and evaluated term-parallel (one lane
// per two-body term, a segmented wave reduction in a fixed order), so a long
// sum never stalls the other 63 lanes.
//
// The same walk serves the count pass (steps 1-2 only), the fill pass and the
// adjoint (step 3 scatters phase * upstream value onto the table).
#include <hip/hip_runtime.h>

#include "ci_internal.h"

namespace ci {

enum { kCount = 0, kFill = 1, kAdjoint = 2 };

constexpr int kWavesPerBlock = 4;
constexpr int kQueue = 128;  // queued multi-term entries per wave

__device__ __forceinline__ int rec_d(uint64_t r) { return (int)((r >> 57) & 3); }
__device__ __forceinline__ int rec_local(uint64_t r) { return (int)(r & kRecLocalMask); }
__device__ __forceinline__ int rec_h1(uint64_t r) { return (int)((r >> 24) & 255); }
__device__ __forceinline__ int rec_p1(uint64_t r) { return (int)((r >> 32) & 255); }
__device__ __forceinline__ int rec_h2(uint64_t r) { return (int)((r >> 40) & 255); }
__device__ __forceinline__ int rec_p2(uint64_t r) { return (int)((r >> 48) & 255); }
__device__ __forceinline__ double rec_sign(uint64_t r) { return ((r >> 56) & 1) ? -1.0 : 1.0; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// LDS writes by one lane become visible to the other lanes of the wavefront
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// largest t in [0, n) with a[t] <= x, for a[0] <= x < a[n], a non-decreasing
__device__ __forceinline__ int seg_search(const int32_t* a, int n, int x)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

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

// Per-wavefront LDS.
struct WaveLds {
    int32_t bstart[65];        // first segment of each target block of the window
    int32_t eoff[65];          // first entry of each segment of the chunk
    uint64_t spr[64];          // proton partner record of each segment
    const uint64_t* slp[64];   // first neutron partner record of each segment
    int64_t scol[64];          // column of local neutron index 0 of each segment
    int32_t qpos[kQueue];      // queued entry: offset from the row's first entry
    uint64_t qpr[kQueue];      //   proton record (self record for no proton move)
    uint64_t qnr[kQueue];      //   neutron record
    int32_t toff[kQueue + 1];  //   first term of each queued entry
    int32_t occ[2 * 64];       // occupied orbits of the row: protons, then neutrons
};

struct RowView {
    const BasisDev* B;
    const float* tbme;  // this basis' table (fill)
    double* gacc;       // this basis' accumulators (adjoint)
    const float* gval;  // upstream values (adjoint)
    int32_t* col;
    float* val;
    int64_t pos0;  // first entry of the row
    int64_t cap;   // end of all entries (no access at or beyond)
    int Z, NN;     // particles
    double spe_sum;
};

// number of two-body terms of a queued entry
__device__ __forceinline__ int queued_terms(const RowView& R, uint64_t pr, uint64_t nr)
{
    const int A = R.Z + R.NN;
    return (rec_d(pr) == 0 && rec_d(nr) == 0) ? A * (A - 1) / 2 : A - 1;
}

// The u-th two-body term of a queued entry: coefficient and table position.
__device__ __forceinline__ int64_t queued_term(const RowView& R, const WaveLds& L, uint64_t pr, uint64_t nr,
                                               int u, double* coef)
{
    const BasisDev& B = *R.B;
    const int Z = R.Z, NN = R.NN;
    const int32_t* oP = L.occ;
    const int32_t* oN = L.occ + Z;
    double s;
    int64_t k;
    if (rec_d(pr) == 1) {  // one proton moved: p (row) -> h (column)
        const int h = rec_h1(pr), p = rec_p1(pr);
        if (u < Z - 1) {  // the u-th proton spectator (the row's protons without p)
            const int kk = (oP[u] >= p) ? oP[u + 1] : oP[u];
            k = tb_index(B, 0, p, kk, h, kk, &s);
        } else {
            const int b = oN[u - (Z - 1)];
            k = tb_index(B, 1, p, b, h, b, &s);
        }
        *coef = rec_sign(pr) * s;
        return k;
    }
    if (rec_d(nr) == 1) {  // one neutron moved
        const int h = rec_h1(nr), p = rec_p1(nr);
        if (u < NN - 1) {
            const int kk = (oN[u] >= p) ? oN[u + 1] : oN[u];
            k = tb_index(B, 2, p, kk, h, kk, &s);
        } else {
            const int a = oP[u - (NN - 1)];
            k = tb_index(B, 1, a, p, a, h, &s);
        }
        *coef = rec_sign(nr) * s;
        return k;
    }
    // diagonal: every occupied pair, pp then nn then pn
    const int npp = Z * (Z - 1) / 2, nnn = NN * (NN - 1) / 2;
    int cls, a, b;
    if (u < npp + nnn) {
        const int32_t* o = (u < npp) ? oP : oN;
        const int X = (u < npp) ? Z : NN;
        int t = (u < npp) ? u : u - npp;
        int x = 0;
        while (t >= X - 1 - x) {
            t -= X - 1 - x;
            x++;
        }
        a = o[x];
        b = o[x + 1 + t];
        cls = (u < npp) ? 0 : 2;
    } else {
        const int t = u - npp - nnn;
        a = oP[t / NN];
        b = oN[t % NN];
        cls = 1;
    }
    k = tb_index(B, cls, a, b, a, b, &s);
    *coef = s;
    return k;
}

// Evaluate (fill) or scatter (adjoint) the queued multi-term entries.
template <int MODE>
__device__ void flush_queue(const RowView& R, WaveLds& L, int qn)
{
    const int lane = threadIdx.x & 63;
    if (qn == 0) return;
    // first term of each queued entry (up to 128 entries: two per lane)
    int tot = 0;
    for (int base = 0; base < qn; base += 64) {
        const int q = base + lane;
        const int t = q < qn ? queued_terms(R, L.qpr[q], L.qnr[q]) : 0;
        const int incl = wave_incl_scan(t);
        L.toff[q + 1] = tot + incl;  // q < kQueue
        if (lane == 0 && base == 0) L.toff[0] = 0;
        tot += __shfl(incl, 63, 64);
    }
    wave_sync();
    double carry = 0.0;
    int carry_q = -1;
    for (int t0 = 0; t0 < tot; t0 += 64) {
        const int t = t0 + lane;
        const bool act = t < tot;
        int q = 0;
        double v = 0.0;
        if (act) {
            q = seg_search(L.toff, qn, t);
            const int u = t - L.toff[q];
            double coef;
            const int64_t k = queued_term(R, L, L.qpr[q], L.qnr[q], u, &coef);
            if (k >= 0) {
                if (MODE == kFill) {
                    v = coef * (double)R.tbme[k];
                } else {
                    const int64_t p = R.pos0 + L.qpos[q];
                    if (p < R.cap) atomicAdd(&R.gacc[k], coef * (double)R.gval[p]);
                }
            }
        }
        if (MODE == kFill) {
            // segmented inclusive scan over the lanes, keyed by q, fixed order
            const int qq = act ? q : 0x7fffffff;
            for (int o = 1; o < 64; o <<= 1) {
                const double vu = __shfl_up(v, o, 64);
                const int qu = __shfl_up(qq, o, 64);
                if (lane >= o && qu == qq) v += vu;
            }
            if (act && q == carry_q) v += carry;
            const int qnext = __shfl_down(qq, 1, 64);
            if (act && (lane == 63 || qnext != qq) && t == L.toff[q + 1] - 1) {
                // the entry's last term: write it
                const int64_t p = R.pos0 + L.qpos[q];
                double x = v;
                if (rec_d(L.qpr[q]) == 0 && rec_d(L.qnr[q]) == 0) x += R.spe_sum;
                if (p < R.cap) R.val[p] = (float)x;
            }
            // an entry cut by the end of the round continues in the next one
            carry = __shfl(v, 63, 64);
            carry_q = __shfl(qq, 63, 64);
        }
    }
    wave_sync();
}

// One row: count (returns the number of entries), fill or adjoint.
template <int MODE>
__device__ int64_t do_row(const BasisDev& B, WaveLds& L, int bi, int64_t r, RowView& R)
{
    const int lane = threadIdx.x & 63;
    const SpeciesDev& SP = B.sp[0];
    const SpeciesDev& SN = B.sp[1];
    const int kp = B.blk_kp[bi], kn = B.blk_kn[bi];
    const int nKn = SN.key_off[kn + 1] - SN.key_off[kn];
    const int ip = (int)(r / nKn), in = (int)(r - (int64_t)ip * nKn);
    const int64_t gP = SP.key_off[kp] + ip;
    const int64_t gN = SN.key_off[kn] + in;
    const int nkp = SP.nk, nkn = SN.nk;
    const uint64_t* P1 = SP.l1 + SP.l1_ptr[gP];
    const uint64_t* P12 = SP.l12 + SP.l12_ptr[gP];
    const int32_t* sP1 = SP.seg1 + gP * (nkp + 1);
    const int32_t* sP12 = SP.seg12 + gP * (nkp + 1);
    const uint64_t* N1 = SN.l1 + SN.l1_ptr[gN];
    const uint64_t* N12 = SN.l12 + SN.l12_ptr[gN];
    const int32_t* sN1 = SN.seg1 + gN * (nkn + 1);
    const int32_t* sN12 = SN.seg12 + gN * (nkn + 1);
    const int self12 = SN.self12[gN];

    if (MODE != kCount) {
        // occupied orbits of the row (for the multi-term entries)
        double e = 0.0;
        if (lane == 0) {
            int t = 0;
            for (int s = 0; s < 2; s++) {
                const uint64_t* w = (s == 0 ? SP.sd + gP * B.W : SN.sd + gN * B.W);
                for (int k = 0; k < B.W; k++) {
                    uint64_t x = w[k];
                    while (x) {
                        const int o = k * 64 + __ffsll((long long)x) - 1;
                        x &= x - 1;
                        L.occ[t++] = o;
                        e += (B.orb_n[o] + 1.5) * B.hw;
                    }
                }
            }
        }
        R.spe_sum = __shfl(e, 0, 64);
        wave_sync();
    }

    int64_t pos = 0;  // entries of the row so far
    int qn = 0;       // queued multi-term entries
    for (int w0 = bi; w0 < B.nblk; w0 += 64) {
        // 1. proton partners of P in each target block of the window
        const int b2 = w0 + lane;
        int np = 0;
        if (b2 < B.nblk) {
            const int kp2 = B.blk_kp[b2];
            np = (B.blk_kn[b2] == kn) ? sP12[kp2 + 1] - sP12[kp2] : sP1[kp2 + 1] - sP1[kp2];
        }
        const int bincl = wave_incl_scan(np);
        L.bstart[lane + 1] = bincl;
        if (lane == 0) L.bstart[0] = 0;
        const int S = __shfl(bincl, 63, 64);
        wave_sync();
        for (int s0 = 0; s0 < S; s0 += 64) {
            // 2. entries of each segment (target block, P')
            const int s = s0 + lane;
            int len = 0;
            uint64_t pr = 0;
            const uint64_t* lp = nullptr;
            int64_t cb = 0;
            if (s < S) {
                const int t = seg_search(L.bstart, 64, s);
                const int bb = w0 + t;
                const int kp2 = B.blk_kp[bb], kn2 = B.blk_kn[bb];
                const bool same_n = (kn2 == kn);
                const int q = s - L.bstart[t];
                pr = same_n ? P12[sP12[kp2] + q] : P1[sP1[kp2] + q];
                const int dp = rec_d(pr), ipp = rec_local(pr);
                cb = B.blk_off[bb] + (int64_t)ipp * (SN.key_off[kn2 + 1] - SN.key_off[kn2]);
                if (bb == bi && ipp < ip) {
                    len = 0;  // lower triangle
                } else if (dp == 2) {
                    len = 1;  // two protons moved: N' = N
                } else if (dp == 1) {
                    lp = N1 + sN1[kn2];
                    len = sN1[kn2 + 1] - sN1[kn2];
                } else {
                    const int k0 = (bb == bi) ? self12 : 0;  // diagonal block: N' >= N
                    lp = N12 + sN12[kn2] + k0;
                    len = sN12[kn2 + 1] - sN12[kn2] - k0;
                }
            }
            const int eincl = wave_incl_scan(len);
            const int T = __shfl(eincl, 63, 64);
            if (MODE == kCount) {
                pos += T;
                continue;
            }
            L.eoff[lane + 1] = eincl;
            if (lane == 0) L.eoff[0] = 0;
            L.spr[lane] = pr;
            L.slp[lane] = lp;
            L.scol[lane] = cb;
            wave_sync();
            // 3. the entries of the chunk, 64 consecutive ones per round
            for (int e0 = 0; e0 < T; e0 += 64) {
                const int e = e0 + lane;
                bool special = false;
                uint64_t qp = 0, qnrec = 0;
                if (e < T) {
                    const int j = seg_search(L.eoff, 64, e);
                    const int k = e - L.eoff[j];
                    const uint64_t prj = L.spr[j];
                    const int dp = rec_d(prj);
                    const int64_t p = R.pos0 + pos + e;
                    int64_t c;
                    int64_t key = -1;
                    double coef = 0.0;
                    if (dp == 2) {  // two protons moved
                        c = L.scol[j] + in;
                        key = tb_index(B, 0, rec_p1(prj), rec_p2(prj), rec_h1(prj), rec_h2(prj), &coef);
                        coef *= rec_sign(prj);
                    } else {
                        const uint64_t nr = L.slp[j][k];
                        c = L.scol[j] + rec_local(nr);
                        const int dn = rec_d(nr);
                        if (dp + dn == 2) {  // one proton and one neutron, or two neutrons, moved
                            if (dp == 1)
                                key = tb_index(B, 1, rec_p1(prj), rec_p1(nr), rec_h1(prj), rec_h1(nr), &coef);
                            else
                                key = tb_index(B, 2, rec_p1(nr), rec_p2(nr), rec_h1(nr), rec_h2(nr), &coef);
                            coef *= rec_sign(prj) * rec_sign(nr);
                        } else {  // diagonal or one nucleon moved: queue
                            special = true;
                            qp = prj;
                            qnrec = nr;
                        }
                    }
                    if (p < R.cap) {
                        if (MODE == kFill) {
                            R.col[p] = (int32_t)c;
                            if (!special) R.val[p] = key >= 0 ? (float)(coef * (double)R.tbme[key]) : 0.0f;
                        } else if (!special && key >= 0) {
                            atomicAdd(&R.gacc[key], coef * (double)R.gval[p]);
                        }
                    }
                }
                const uint64_t m = __ballot(special);
                if (m) {
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                    if (special) {
                        L.qpos[qn + rank] = (int32_t)(pos + e);
                        L.qpr[qn + rank] = qp;
                        L.qnr[qn + rank] = qnrec;
                    }
                    qn += __popcll(m);
                    wave_sync();
                    if (qn > kQueue - 64) {  // room for one more round
                        flush_queue<MODE>(R, L, qn);
                        qn = 0;
                    }
                }
            }
            pos += T;
            wave_sync();
        }
    }
    if (MODE != kCount) flush_queue<MODE>(R, L, qn);
    return pos;
}

// One wavefront per row; the rows of all bases are numbered consecutively.
template <int MODE>
__global__ void __launch_bounds__(64 * kWavesPerBlock)
    row_kernel(const BasisDev* __restrict__ bases, int nb, const int64_t* __restrict__ basis_row0,
               int64_t nrows, const float* __restrict__ tbme, int64_t* __restrict__ row_ptr, int64_t nrp,
               int32_t* __restrict__ col, float* __restrict__ val, const float* __restrict__ gval,
               double* __restrict__ gacc)
{
    __shared__ WaveLds lds[kWavesPerBlock];
    const int wid = uniform(threadIdx.x >> 6);
    const int64_t grow = (int64_t)blockIdx.x * kWavesPerBlock + wid;
    if (grow >= nrows) return;
    // basis of the row (few bases: linear search)
    int b = 0;
    while (b + 1 < nb && basis_row0[b + 1] <= grow) b++;
    b = uniform(b);
    const BasisDev& B = bases[b];
    const int64_t i = grow - basis_row0[b];
    // block of the row
    int lo = 0, hi = B.nblk;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (B.blk_off[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int bi = uniform(lo);
    RowView R;
    R.B = &B;
    R.tbme = tbme ? tbme + B.tbme0 : nullptr;
    R.gacc = gacc ? gacc + B.tbme0 : nullptr;
    R.gval = gval;
    R.col = col;
    R.val = val;
    R.Z = B.Z;
    R.NN = B.NN;
    R.spe_sum = 0.0;
    if (MODE == kCount) {
        R.pos0 = 0;
        R.cap = 0;
        const int64_t n = do_row<kCount>(B, lds[wid], bi, i - B.blk_off[bi], R);
        if ((threadIdx.x & 63) == 0) row_ptr[B.row0 + i + 1] = n;
    } else {
        R.pos0 = uniform64(row_ptr[B.row0 + i]);
        R.cap = uniform64(row_ptr[nrp - 1]);  // the entries of all bases end here
        do_row<MODE>(B, lds[wid], bi, i - B.blk_off[bi], R);
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

hipError_t launch_inclusive_scan(int64_t* x, int64_t n, int64_t* tmp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t nbk = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_block_sums, dim3((unsigned)nbk), dim3(kScanThreads), 0, s, x, n, tmp);
    hipLaunchKernelGGL(scan_sums_exclusive, dim3(1), dim3(kScanThreads), 0, s, tmp, nbk);
    hipLaunchKernelGGL(scan_apply, dim3((unsigned)nbk), dim3(kScanThreads), 0, s, x, n, tmp);
    return hipGetLastError();
}

__global__ void copy_i64(const int64_t* __restrict__ src, int64_t* __restrict__ dst) { *dst = *src; }

hipError_t launch_copy_i64(const int64_t* src, int64_t* dst, hipStream_t s)
{
    hipLaunchKernelGGL(copy_i64, dim3(1), dim3(1), 0, s, src, dst);
    return hipGetLastError();
}

hipError_t launch_count(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                        int64_t* row_ptr, int64_t nrp, const int64_t* seg_first, int64_t* scan_tmp,
                        hipStream_t s)
{
    if (nrows > 0)
        hipLaunchKernelGGL(row_kernel<kCount>, dim3(grid_for(nrows, kWavesPerBlock)),
                           dim3(64 * kWavesPerBlock), 0, s, bases, nb, basis_row0, nrows, nullptr, row_ptr,
                           nrp, nullptr, nullptr, nullptr, nullptr);
    // the first slot of each basis' segment holds 0 before the scan, so the
    // inclusive scan leaves there the number of entries of the bases before it
    hipLaunchKernelGGL(zero_i64_at, dim3(grid_for(nb, 256)), dim3(256), 0, s, row_ptr, seg_first, nb);
    return launch_inclusive_scan(row_ptr, nrp, scan_tmp, s);
}

hipError_t launch_nnz(const int64_t* row_ptr, const int64_t* first, const int64_t* last, int64_t* nnz,
                      int n, hipStream_t s)
{
    hipLaunchKernelGGL(nnz_of_bases, dim3(grid_for(n, 256)), dim3(256), 0, s, row_ptr, first, last, nnz, n);
    return hipGetLastError();
}

hipError_t launch_fill(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                       const float* tbme, const int64_t* row_ptr, int64_t nrp, int32_t* col, float* val,
                       hipStream_t s)
{
    if (nrows > 0)
        hipLaunchKernelGGL(row_kernel<kFill>, dim3(grid_for(nrows, kWavesPerBlock)), dim3(64 * kWavesPerBlock),
                           0, s, bases, nb, basis_row0, nrows, tbme, const_cast<int64_t*>(row_ptr), nrp, col,
                           val, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_vjp(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                      const int64_t* row_ptr, int64_t nrp, const float* gval, float* gtbme, double* gacc,
                      int64_t ntbme, hipStream_t s)
{
    const unsigned gz = grid_for(ntbme, 256) < 4096 ? grid_for(ntbme, 256) : 4096;
    if (ntbme > 0) hipLaunchKernelGGL(fill_f64, dim3(gz), dim3(256), 0, s, gacc, ntbme, 0.0);
    if (nrows > 0)
        hipLaunchKernelGGL(row_kernel<kAdjoint>, dim3(grid_for(nrows, kWavesPerBlock)),
                           dim3(64 * kWavesPerBlock), 0, s, bases, nb, basis_row0, nrows, nullptr,
                           const_cast<int64_t*>(row_ptr), nrp, nullptr, nullptr, gval, gacc);
    if (ntbme > 0) hipLaunchKernelGGL(f64_to_f32, dim3(gz), dim3(256), 0, s, gacc, gtbme, ntbme);
    return hipGetLastError();
}

}  // namespace ci
