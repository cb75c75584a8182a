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

#include <atomic>

#include "ci_internal.h"

namespace ci {

enum { kCount = 0, kFill = 1, kAdjoint = 2 };

constexpr int kWavesPerBlock = 4;
constexpr int kQueue = 96;  // queued multi-term entries per wave

__device__ __forceinline__ int rec_d(uint64_t r) { return (int)((r >> 57) & 3); }
__device__ __forceinline__ int rec_local(uint64_t r) { return (int)(r & kRecLocalMask); }
__device__ __forceinline__ int rec_h1(uint64_t r) { return (int)((r >> 24) & 255); }
__device__ __forceinline__ int rec_p1(uint64_t r) { return (int)((r >> 32) & 255); }
__device__ __forceinline__ int rec_h2(uint64_t r) { return (int)((r >> 40) & 255); }
__device__ __forceinline__ int rec_p2(uint64_t r) { return (int)((r >> 48) & 255); }
__device__ __forceinline__ double rec_sign(uint64_t r) { return ((r >> 56) & 1) ? -1.0 : 1.0; }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Pointers read from the descriptors are generic; accessing them through the
// global address space gives global_load instead of flat_load (a flat load
// also counts against the LDS wait counter and would stall every LDS access).
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> glb(const T* p)
{
    return (gptr<T>)p;
}
template <typename T>
using gmut = __attribute__((address_space(1))) T*;
// relaxed device-scope add of a signed 64-bit integer (two's complement) in L2
__device__ __forceinline__ void atomic_add_i64(gmut<unsigned long long> p, int64_t v)
{
    __hip_atomic_fetch_add(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ gmut<T> glbw(T* p)
{
    return (gmut<T>)p;
}
template <typename T>
using lptr = __attribute__((address_space(3))) T*;

// Element i of an array whose base is uniform (scalar registers), addressed
// by a 32-bit byte offset: the load or store then takes the base + offset
// form, with no 64-bit address arithmetic per lane (i * sizeof(T) < 2^32).
template <typename T>
__device__ __forceinline__ T ld32(const T* base, uint32_t i)
{
    return *(gptr<T>)((const __attribute__((address_space(1))) char*)base + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st32(T* base, uint32_t i, T v)
{
    *(gmut<T>)((__attribute__((address_space(1))) char*)base + i * (uint32_t)sizeof(T)) = v;
}

typedef int i32x4 __attribute__((ext_vector_type(4)));  // a BlockInfo record

// The index tables and row_ptr do not change while a row kernel runs, so the
// row-uniform reads of them go through the constant address space: the
// compiler then issues scalar loads (scalar cache) instead of vector loads,
// which would all pass through the vector memory pipeline.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> cst(const T* p)
{
    return (cptr<T>)p;
}

// Adjoint: the rows of a workgroup scatter into a shared LDS table first
// (open addressing on the global table position, int32 fixed-point partial
// sums), and each occupied slot is added to the int64 accumulator once at the
// end.  Table keys
// repeat across consecutive rows (the same proton move for every row of one
// proton determinant, and overlapping neutron moves), so the number of
// device-scope atomics drops by that reuse factor.  A key that finds no slot
// within kAdjProbes probes goes to the accumulator directly.
// Two workgroup shapes: the adjoint that walks the partner lists has work to
// overlap with its device-scope atomics and runs best at 8 wavefronts and a
// 4096-slot table (three workgroups per CU); the adjoint that reads stored
// words has little, and runs best with fewer atomics: 16 wavefronts sharing a
// 16384-slot table (128 KiB of the CU's 160 KiB, one workgroup per CU).
constexpr int kAdjWaves = 8;
constexpr int kAdjSlotBits = 12;
constexpr int kAdjKeysWaves = 16;
constexpr int kAdjKeysSlotBits = 14;
constexpr int kAdjProbes = 16;
constexpr uint32_t kAdjEmpty = 0xffffffffu;

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Workgroups of a launch are dealt to the 8 XCDs of the device in turn
// (workgroup g runs on XCD g mod 8), and each XCD has its own L2.  With
// this mapping XCD x runs the logical workgroups of one contiguous eighth of
// the grid, so the rows (or tiles) that one L2 serves at a time are
// neighbours and share their partner lists.  A bijection on [0, n).
__device__ __forceinline__ int64_t xcd_contiguous(int64_t g, int64_t n)
{
    constexpr int kXcds = 8;
    const int64_t x = g % kXcds, slot = g / kXcds, q = n / kXcds, r = n % kXcds;
    return x < r ? x * (q + 1) + slot : r * (q + 1) + (x - r) * q + slot;
}

// LDS writes by one lane become visible to the other lanes of the wavefront
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (no LDS traffic).
__device__ __forceinline__ int wave_incl_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
    return v;
}

__device__ __forceinline__ int lane63(int v) { return __builtin_amdgcn_readlane(v, 63); }

// Inclusive running maximum over the 64 lanes of values >= 0, DPP as above
// (a lane with no source reads 0, which changes no maximum).
__device__ __forceinline__ int wave_incl_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true));  // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true));  // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true));  // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true));  // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, true));  // row_bcast:15 into rows 1, 3
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, true));  // row_bcast:31 into rows 2, 3
    return v;
}

// FP64 sum over the 64 lanes in a fixed butterfly order (every lane ends with
// the same value, bit for bit, whatever the launch shape)
__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// largest t in [0, 64) with a[t] <= x, for a[0] <= x < a[64], a non-decreasing
__device__ __forceinline__ int seg_search64(const int32_t* a, int x)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (a[lo + step] <= x) lo += step;
    return lo;
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
// species-local orbits, for ordered pairs (a < b and c < d for pp and nn; a,
// c protons and b, d neutrons for pn).  -1 if a pair is outside the table.
__device__ __forceinline__ int tb_pos(const BasisDev& B, int cls, int a, int b, int c, int d)
{
    // 32-bit unsigned offsets from the table's base (an SGPR pair): the loads
    // take their address as base + offset with no 64-bit arithmetic per lane
    const uint32_t n = (uint32_t)B.nsps, o = (uint32_t)cls * n * n;
    const uint64_t e1 = ld32(B.pair, o + (uint32_t)a * n + (uint32_t)b);
    const uint64_t e2 = ld32(B.pair, o + (uint32_t)c * n + (uint32_t)d);
    const uint32_t l1 = (uint32_t)e1, l2 = (uint32_t)e2;
    if (e1 == kNoPair64 || e2 == kNoPair64 || (l1 >> 16) != (l2 >> 16)) return -1;
    const bool first = (l1 & 0xffff) <= (l2 & 0xffff);
    return (int)((first ? (uint32_t)(e1 >> 32) : (uint32_t)(e2 >> 32)) + (first ? (l2 & 0xffff) : (l1 & 0xffff)));
}

// Same for pairs in any order: each swap inside a pp or nn pair flips the sign.
__device__ __forceinline__ int tb_pos_any(const BasisDev& B, int cls, int a, int b, int c, int d, bool* neg)
{
    bool ng = false;
    if (cls != 1) {
        if (a > b) { const int t = a; a = b; b = t; ng = !ng; }
        if (c > d) { const int t = c; c = d; d = t; ng = !ng; }
    }
    *neg = ng;
    return tb_pos(B, cls, a, b, c, d);
}

__device__ __forceinline__ bool rec_neg(uint64_t r) { return (r >> 56) & 1; }

// Per-wavefront LDS.
// Per-wavefront LDS: the queue of multi-term entries and the row's occupied
// orbits.  The per-block and per-segment values of the walk stay in registers
// (lane t holds block / segment t) and are read across lanes with ds_bpermute.
struct WaveLds {
    int32_t qpos[kQueue];  // offset from the row's first entry
    uint32_t qrec[kQueue]; // kind (0 diagonal, 1 one proton moved, 2 one neutron moved) | h << 8 | p << 16 | neg << 24
    union {
        int32_t toff[kQueue + 1];  // first term of each queued entry
        double tsum[64];           // fill: one term per lane, summed by the entry's first lane
    };
    int32_t mark[64];  // load balancing: mark[x] = the lane whose item starts at x of the round
    uint8_t occ[128];  // occupied orbits of the row: protons, then neutrons
};

// Load-balanced search: lanes hold consecutive non-overlapping ranges
// [start, start + len) of a sequence (ascending in the lane index); for the
// round of 64 items [x0, x0 + 64) every lane x learns the lane whose range holds
// item x0 + x.  A lane whose range starts inside the round writes its index at
// that offset of mark[], then a running maximum carries each owner over the
// items of its range.  carry: the owner of item x0 - 1 (-1 before the first
// round); mark[] must hold values <= carry outside this round's starts (-1
// after clear_marks, then the owners of earlier rounds).  Returns the owner,
// in [0, 64) for every item of the sequence.
__device__ __forceinline__ void clear_marks(WaveLds& L)
{
    L.mark[threadIdx.x & 63] = -1;
    wave_sync();
}
__device__ __forceinline__ int owner_of(WaveLds& L, int start, int len, int x0, int* carry)
{
    const int lane = threadIdx.x & 63;
    const int rel = start - x0;
    if (len > 0 && rel >= 0 && rel < 64) L.mark[rel] = lane;
    wave_sync();
    // owners are shifted by one so that "none" is 0, the identity of the maximum
    const int o = wave_incl_max(max(L.mark[lane], *carry) + 1);
    *carry = __builtin_amdgcn_readlane(o, 63) - 1;
    wave_sync();
    return o > 0 ? o - 1 : 0;
}

__device__ __forceinline__ int q_kind(uint32_t q) { return (int)(q & 3); }
__device__ __forceinline__ int q_h(uint32_t q) { return (int)((q >> 8) & 255); }
__device__ __forceinline__ int q_p(uint32_t q) { return (int)((q >> 16) & 255); }
__device__ __forceinline__ bool q_neg(uint32_t q) { return (q >> 24) & 1; }

// value v of lane l (every lane of the wavefront must be active)
__device__ __forceinline__ int lane_read(int v, int l) { return __builtin_amdgcn_ds_bpermute(l << 2, v); }
__device__ __forceinline__ uint64_t lane_read64(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)lane_read((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)lane_read((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// largest t in [0, 64) with start(t) <= x, where lane t holds start(t),
// non-decreasing in t, and start(0) <= x (every lane active)
__device__ __forceinline__ int lane_search64(int start, int x)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (lane_read(start, lo + step) <= x) lo += step;
    return lo;
}

// Word stored per entry for the adjoint: a single two-body term holds its
// table position in the low 30 bits (kKeyNone: no table element, the entry is
// 0) and its sign in bit 30; a multi-term entry (diagonal, one nucleon moved)
// sets bit 31 and holds its queue record in the low 25 bits.
constexpr uint32_t kKeySpecial = 0x80000000u;
constexpr uint32_t kKeyNeg = 0x40000000u;
constexpr uint32_t kKeyPos = 0x3fffffffu;
constexpr uint32_t kKeyNone = 0x3fffffffu;

struct RowView {
    const BasisDev* B;
    const float* tbme;  // this basis' table (fill)
    unsigned long long* gacc;  // this basis' int64 fixed-point accumulators (adjoint)
    int64_t tbme0;      // this basis' first table position in the batch
    // LDS accumulator table of the workgroup (adjoint); used only when
    // use_table is set (an LDS address can be 0, so no null test on it)
    lptr<uint32_t> hkey;
    lptr<int32_t> hval;
    bool use_table;
    int hbits;  // the table has 1 << hbits slots
    int qshift; // adjoint contribution g counts as the integer rint(g * 2^qshift)
    const float* gval;  // upstream values (adjoint)
    int32_t* col;
    float* val;
    uint32_t* keys;  // one word per stored entry (written by the fill, read by the adjoint), or null
    int64_t pos0;  // first entry of the row
    int64_t cap;   // end of all entries (no access at or beyond)
    int Z, NN;     // particles
    bool full;     // both triangles (every column), not only j >= i
    double spe_sum;
};

// Adjoint contribution g to table position k of the row's basis, in fixed
// point: q = rint(g * 2^qshift), an exact power-of-two scaling and one
// rounding.  Integer sums do not depend on their order, so the gradient is the
// same bit for bit whatever the tile shape, the flush and the order in which
// wavefronts and atomics meet.  The shift is chosen from max |G| and the rows
// of a tile so that a tile's sum in an int32 LDS slot cannot overflow: a row
// adds at most one contribution to any table position (its moves are distinct
// and a move and its reverse cannot both start from one determinant), so a slot
// receives at most one per row of the tile.  LDS sums use the native integer
// add (this device runs ds_add_f32 at 0.33 lane-operations per CU cycle on
// random addresses of a 4096-word table, far below its integer atomics).
__device__ __forceinline__ void adj_add(const RowView& R, int k, float g)
{
    const int32_t q = (int32_t)__float2int_rn(ldexpf(g, R.qshift));
    if (R.use_table) {
        const uint32_t gk = (uint32_t)(R.tbme0 + k);
        uint32_t s = (gk * 2654435761u) >> (32 - R.hbits);
        for (int t = 0; t < kAdjProbes; t++) {
            // claim an empty slot, or learn which key holds it (one LDS round trip)
            uint32_t cur = kAdjEmpty;
            const bool won = __hip_atomic_compare_exchange_strong(R.hkey + s, &cur, gk, __ATOMIC_RELAXED,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (won || cur == gk) {
                __hip_atomic_fetch_add(R.hval + s, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                return;
            }
            s = (s + 1) & ((1u << R.hbits) - 1);
        }
    }
    atomic_add_i64(glbw(R.gacc) + k, (int64_t)q);
}

// An int64 fixed-point sum (two's complement in the word) as FP32.
__device__ __forceinline__ float fixed_to_f32(unsigned long long v, int qshift)
{
    return (float)ldexp((double)(int64_t)v, -qshift);
}

// number of terms of a queued entry: two-body terms, plus the one-body
// kinetic term of a one-nucleon difference when the problem has it
__device__ __forceinline__ int queued_terms(const RowView& R, uint32_t q)
{
    const int A = R.Z + R.NN;
    return q_kind(q) == 0 ? A * (A - 1) / 2 : A - 1 + R.B->kinetic;
}

// Off-diagonal oscillator kinetic element between species-local orbits p != h:
// (hw/2) sqrt((n+1)(n+l+3/2)) for radial quantum numbers n, n+1 of the same
// (l, j, m), else 0.
__device__ __forceinline__ double kinetic_offdiag(const BasisDev& B, int p, int h)
{
    const int qp = glb(B.orb_qn)[p], qh = glb(B.orb_qn)[h];
    if ((qp >> 8) != (qh >> 8)) return 0.0;  // l, 2j, 2m differ
    const int np = qp & 255, nh = qh & 255, l = (qp >> 8) & 255;
    const int lo = np < nh ? np : nh, hi = np < nh ? nh : np;
    if (hi != lo + 1) return 0.0;
    return 0.5 * B.hw * sqrt((double)(lo + 1) * ((double)lo + l + 1.5));
}

// The u-th two-body term of a queued entry: table position and sign.
// The u-th term: table position (or -1) and sign; *ob receives the one-body
// value of the kinetic term (0 for two-body terms).
__device__ __forceinline__ int queued_term(const RowView& R, const WaveLds& L, uint32_t q, int u, bool* neg,
                                           double* ob)
{
    *ob = 0.0;
    if (q_kind(q) != 0 && u == R.Z + R.NN - 1) {  // the kinetic term a+_p a_h
        *neg = q_neg(q);
        *ob = kinetic_offdiag(*R.B, q_p(q), q_h(q));
        return -1;
    }
    const BasisDev& B = *R.B;
    const int Z = R.Z, NN = R.NN;
    const uint8_t* oP = L.occ;
    const uint8_t* oN = L.occ + Z;
    bool s;
    int k;
    if (q_kind(q) == 1) {  // one proton moved: p (row) -> h (column)
        const int h = q_h(q), p = q_p(q);
        if (u < Z - 1) {  // the u-th proton spectator (the row's protons without p)
            const int kk = (oP[u] >= p) ? oP[u + 1] : oP[u];
            k = tb_pos_any(B, 0, p, kk, h, kk, &s);
        } else {
            const int b = oN[u - (Z - 1)];
            k = tb_pos_any(B, 1, p, b, h, b, &s);
        }
        *neg = s ^ q_neg(q);
        return k;
    }
    if (q_kind(q) == 2) {  // one neutron moved
        const int h = q_h(q), p = q_p(q);
        if (u < NN - 1) {
            const int kk = (oN[u] >= p) ? oN[u + 1] : oN[u];
            k = tb_pos_any(B, 2, p, kk, h, kk, &s);
        } else {
            const int a = oP[u - (NN - 1)];
            k = tb_pos_any(B, 1, a, p, a, h, &s);
        }
        *neg = s ^ q_neg(q);
        return k;
    }
    // diagonal: every occupied pair, pp then nn then pn (all ordered)
    const int npp = Z * (Z - 1) / 2, nnn = NN * (NN - 1) / 2;
    int cls, a, b;
    if (u < npp + nnn) {
        const uint8_t* o = (u < npp) ? oP : oN;
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
    *neg = false;
    return tb_pos(B, cls, a, b, a, b);
}

// The u-th term of a queued one-nucleon difference (kind 1: a proton moved,
// kind 2: a neutron moved; p the row's orbit, h the column's): the spectators
// of the moved nucleon's own species in ascending order, then those of the
// other species; with the kinetic term, a last one-body term.  Written with
// selects so that the lanes of one round, whatever their kinds, take one path.
__device__ __forceinline__ int single_term(const RowView& R, const WaveLds& L, uint32_t q, int u, bool* neg,
                                           double* ob)
{
    const int Z = R.Z, NN = R.NN;
    const bool prot = q_kind(q) == 1;
    const int h = q_h(q), p = q_p(q);
    *ob = 0.0;
    if (u == Z + NN - 1) {  // the kinetic term a+_p a_h
        *neg = q_neg(q);
        *ob = kinetic_offdiag(*R.B, p, h);
        return -1;
    }
    const int X = prot ? Z : NN;
    const uint8_t* own = prot ? L.occ : L.occ + Z;
    const uint8_t* oth = prot ? L.occ + Z : L.occ;
    int cls, a, b, c, d;
    if (u < X - 1) {  // same species: the spectator kk, skipping p
        const int kk = own[u] >= p ? own[u + 1] : own[u];
        cls = prot ? 0 : 2;
        a = p;
        b = kk;
        c = h;
        d = kk;
    } else {  // the other species: proton first in a proton-neutron pair
        const int o = oth[u - (X - 1)];
        cls = 1;
        a = prot ? p : o;
        b = prot ? o : p;
        c = prot ? h : o;
        d = prot ? o : h;
    }
    bool s;
    const int k = tb_pos_any(*R.B, cls, a, b, c, d, &s);
    *neg = s ^ q_neg(q);
    return k;
}

// A queue that holds only one-nucleon differences (the walk treats the
// diagonal on its own), each with the same number of terms nt = A - 1 (+1
// with the kinetic term).  A round takes floor(64 / nt) entries and lane
// k * nt + u takes term u of entry k.  Fill: the entry's first lane sums its nt
// terms from LDS in order (FP64, rounded once).  Adjoint: every term lane adds
// phase * G of its entry to the term's table position.  No search, one path.
template <int MODE>
__device__ void flush_singles(const RowView& R, WaveLds& L, int qn)
{
    const int lane = threadIdx.x & 63;
    const int nt = R.Z + R.NN - 1 + R.B->kinetic;
    if (nt == 0) {  // a single nucleon and no kinetic term: the difference is 0
        if (MODE == kFill)
            for (int q = lane; q < qn; q += 64) {
                const int64_t p = R.pos0 + L.qpos[q];
                if (p < R.cap) glbw(R.val)[p] = 0.0f;
            }
        wave_sync();
        return;
    }
    const int per = 64 / nt;
    const float inv = 1.0f / (float)nt;
    const int k = (int)(((float)lane + 0.5f) * inv);  // exact: the fraction stays >= 0.5 / 64 from an integer
    const int u = lane - k * nt;
    for (int q0 = 0; q0 < qn; q0 += per) {
        const int q = q0 + k;
        const bool act = k < per && q < qn;
        if (MODE == kAdjoint) {
            if (act) {
                bool neg;
                double ob;
                const int kk = single_term(R, L, L.qrec[q], u, &neg, &ob);
                const int64_t p = R.pos0 + L.qpos[q];
                if (kk >= 0 && p < R.cap) {
                    const float g = glb(R.gval)[p];
                    adj_add(R, kk, neg ? -g : g);
                }
            }
            continue;
        }
        double v = 0.0;
        if (act) {
            bool neg;
            double ob;
            const int kk = single_term(R, L, L.qrec[q], u, &neg, &ob);
            const double x = kk >= 0 ? (double)glb(R.tbme)[kk] : ob;
            v = neg ? -x : x;
        }
        L.tsum[lane] = v;
        wave_sync();
        if (act && u == 0) {
            double sum = 0.0;
            for (int i = 0; i < nt; i++) sum += L.tsum[lane + i];
            const int64_t p = R.pos0 + L.qpos[q];
            if (p < R.cap) glbw(R.val)[p] = (float)sum;
        }
        wave_sync();
    }
}

// Evaluate (fill) or scatter (adjoint) the queued multi-term entries.
// SINGLES: the queue holds no diagonal entry (the walk's own queue).
template <int MODE, bool SINGLES>
__device__ void flush_queue(const RowView& R, WaveLds& L, int qn)
{
    const int lane = threadIdx.x & 63;
    if (qn == 0) return;
    if (SINGLES && R.Z + R.NN - 1 + R.B->kinetic <= 64) {
        flush_singles<MODE>(R, L, qn);
        return;
    }
    // first term of each queued entry
    int tot = 0;
    for (int base = 0; base < qn; base += 64) {
        const int q = base + lane;
        const int t = q < qn ? queued_terms(R, L.qrec[q]) : 0;
        if (MODE == kFill && q < qn && t == 0) {
            // no terms (a single nucleon): the diagonal is its single-particle
            // energy, a one-nucleon difference is 0
            const int64_t p = R.pos0 + L.qpos[q];
            if (p < R.cap) glbw(R.val)[p] = q_kind(L.qrec[q]) == 0 ? (float)R.spe_sum : 0.0f;
        }
        const int incl = wave_incl_scan(t);
        if (q < kQueue) L.toff[q + 1] = tot + incl;
        if (lane == 0 && base == 0) L.toff[0] = 0;
        tot += lane63(incl);
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
            bool neg;
            double ob;
            const int k = queued_term(R, L, L.qrec[q], t - L.toff[q], &neg, &ob);
            if (MODE == kFill && k < 0) v = neg ? -ob : ob;
            if (k >= 0) {
                if (MODE == kFill) {
                    const double x = (double)glb(R.tbme)[k];
                    v = neg ? -x : x;
                } else {
                    const int64_t p = R.pos0 + L.qpos[q];
                    if (p < R.cap) {
                        const float g = glb(R.gval)[p];
                        adj_add(R, k, neg ? -g : g);
                    }
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
                if (q_kind(L.qrec[q]) == 0) x += R.spe_sum;
                if (p < R.cap) glbw(R.val)[p] = (float)x;
            }
            // an entry cut by the end of the round continues in the next one
            carry = __shfl(v, 63, 64);
            carry_q = __shfl(qq, 63, 64);
        }
    }
    wave_sync();
}

// The row's diagonal entry: fill, its value, the single-particle sum plus every
// occupied pair V_{ab,ab} (pp, nn, pn), one lane per pair, summed in FP64 in a
// fixed order and rounded once; adjoint, G of the entry added to every
// occupied pair's table position.  Lane u < Z(Z-1)/2 takes proton pair u in
// colex order (u = y(y-1)/2 + x, x < y), the next N(N-1)/2 lanes the neutron
// pairs, the last Z*N lanes the proton-neutron pairs.
template <int MODE>
__device__ void row_diagonal(const RowView& R, const WaveLds& L, int64_t p)
{
    const int lane = threadIdx.x & 63;
    const BasisDev& B = *R.B;
    const int Z = R.Z, NN = R.NN;
    const int npp = Z * (Z - 1) / 2, nnn = NN * (NN - 1) / 2, tot = npp + nnn + Z * NN;
    const float g = (MODE == kAdjoint && p < R.cap) ? glb(R.gval)[p] : 0.0f;
    double acc = 0.0;
    for (int u0 = 0; u0 < tot; u0 += 64) {
        const int u = u0 + lane;
        if (u < tot) {
            int cls, a, b;
            if (u < npp + nnn) {
                const bool pp = u < npp;
                const int t = pp ? u : u - npp;
                int y = (int)(0.5f * (1.0f + sqrtf(1.0f + 8.0f * (float)t)));
                while (y * (y - 1) / 2 > t) y--;
                while ((y + 1) * y / 2 <= t) y++;
                const int x = t - y * (y - 1) / 2;
                const uint8_t* o = pp ? L.occ : L.occ + Z;
                a = o[x];
                b = o[y];
                cls = pp ? 0 : 2;
            } else {
                const int t = u - npp - nnn;
                const int ia = t / NN;
                a = L.occ[ia];
                b = L.occ[Z + (t - ia * NN)];
                cls = 1;
            }
            const int k = tb_pos(B, cls, a, b, a, b);
            if (MODE == kFill && k >= 0) acc += (double)glb(R.tbme)[k];
            if (MODE == kAdjoint && k >= 0 && p < R.cap) adj_add(R, k, g);
        }
    }
    if (MODE == kFill) {
        acc = wave_sum_f64(acc);
        if (lane == 0 && p < R.cap) glbw(R.val)[p] = (float)(acc + R.spe_sum);
    }
}

// Occupied orbits of row (gP, gN) into L.occ, for the multi-term entries:
// lane j < 2W holds determinant word j (protons, then neutrons), a wave scan
// gives each word's first slot in occ, and (spe: for the fill's values) the
// shells of the occupied orbits give the single-particle sum.
__device__ void row_occ(const BasisDev& B, WaveLds& L, RowView& R, int gP, int gN, bool spe)
{
    const int lane = threadIdx.x & 63;
    const SpeciesDev& SP = B.sp[0];
    const SpeciesDev& SN = B.sp[1];
    const int W = B.W;
    uint64_t word = 0;
    if (lane < 2 * W)
        word = lane < W ? glb(SP.sd)[(int64_t)gP * W + lane] : glb(SN.sd)[(int64_t)gN * W + (lane - W)];
    const int cnt = __popcll(word);
    int t = wave_incl_scan(cnt) - cnt;
    const int obase = (lane < W ? lane : lane - W) * 64;
    for (uint64_t x = word; x; x &= x - 1) L.occ[t++] = (uint8_t)(obase + __ffsll((long long)x) - 1);
    wave_sync();
    if (!spe) return;
    const int A = R.Z + R.NN;
    int shells = 0;
    for (int j0 = 0; j0 < A; j0 += 64) {
        const int j = j0 + lane;
        shells += lane63(wave_incl_scan(j < A ? glb(B.orb_n)[L.occ[j]] : 0));
    }
    // oscillator energies (N + 3/2) hw; with the kinetic term the diagonal of
    // T, (hw/2)(N + 3/2)
    R.spe_sum = ((double)shells + 1.5 * A) * B.hw * (B.kinetic ? 0.5 : 1.0);
}

// One row: count (returns the number of entries), fill or adjoint.
template <int MODE>
__device__ int64_t do_row(const BasisDev& B, WaveLds& L, int bi, int r, RowView& R)
{
    const int lane = threadIdx.x & 63;
    const SpeciesDev& SP = B.sp[0];
    const SpeciesDev& SN = B.sp[1];
    const cptr<int32_t> pkoff = cst(SP.key_off), nkoff = cst(SN.key_off);
    const int kp = uniform(cst(B.blk_kp)[bi]), kn = uniform(cst(B.blk_kn)[bi]);
    const int nKn = nkoff[kn + 1] - nkoff[kn];
    const int ip = uniform(r / nKn), in = uniform(r - ip * nKn);
    const int gP = uniform(pkoff[kp] + ip);
    const int gN = uniform(nkoff[kn] + in);
    const int nkp = SP.nk, nkn = SN.nk;
    const gptr<uint64_t> P1 = glb(SP.l1 + cst(SP.l1_ptr)[gP]);
    const gptr<uint64_t> P12 = glb(SP.l12 + cst(SP.l12_ptr)[gP]);
    const gptr<int32_t> sP1 = glb(SP.seg1 + (int64_t)gP * (nkp + 1));
    const gptr<int32_t> sP12 = glb(SP.seg12 + (int64_t)gP * (nkp + 1));
    const gptr<uint64_t> N1 = glb(SN.l1 + cst(SN.l1_ptr)[gN]);
    const gptr<uint64_t> N12 = glb(SN.l12 + cst(SN.l12_ptr)[gN]);
    const gptr<int32_t> sN1 = glb(SN.seg1 + (int64_t)gN * (nkn + 1));
    const gptr<int32_t> sN12 = glb(SN.seg12 + (int64_t)gN * (nkn + 1));
    const int self12 = uniform(cst(SN.self12)[gN]);

    if (MODE != kCount) row_occ(B, L, R, gP, gN, MODE == kFill);

    int64_t pos = 0;  // entries of the row so far
    int qn = 0;       // queued multi-term entries
    int diag_at = -1; // position of the diagonal entry in the row
    for (int w0 = R.full ? 0 : bi; w0 < B.nblk; w0 += 64) {
        // 1. lane t: target block w0 + t of the window: proton partners of P,
        //    the row's neutron partners, column base
        const int b2 = w0 + lane;
        int np = 0, bp = 0, bcol = 0, bstr = 0, bn1 = 0, bl1 = 0, bn12 = 0, bl12 = 0;
        int64_t blen = 0;  // count pass: entries of the lane's block (other blocks than the row's)
        if (b2 < B.nblk) {
            const i32x4 bk = glb((const i32x4*)B.blk)[b2];  // one 16-byte load
            const int kp2 = bk.x, kn2 = bk.y;
            const bool same_n = (kn2 == kn);
            const int ps = same_n ? sP12[kp2] : sP1[kp2];
            np = (same_n ? sP12[kp2 + 1] : sP1[kp2 + 1]) - ps;
            bp = ps | (same_n ? (int)0x80000000 : 0);
            bcol = bk.z;  // first row of the block
            bstr = bk.w;  // |Kn'|
            bn1 = sN1[kn2];
            bl1 = sN1[kn2 + 1] - bn1;
            bn12 = sN12[kn2] + (b2 == bi && !R.full ? self12 : 0);  // diagonal block: N' >= N
            bl12 = sN12[kn2 + 1] - bn12;
            // a block with another neutron key needs a neutron partner of N in it
            // (d <= 1 for a moved proton, d <= 2 for P' = P): otherwise every
            // segment of the block is empty
            if (!same_n && bl1 == 0 && (kp2 != kp || bl12 == 0)) np = 0;
            if (MODE == kCount && (b2 != bi || R.full)) {
                // entries of a block other than the row's own, from the per-key
                // counts: P' = P gives bl12, every one-proton move bl1, every
                // two-proton move (same neutron key only) one entry
                const int d0 = kp2 == kp ? 1 : 0;
                const int c1 = sP1[kp2 + 1] - sP1[kp2];  // d <= 1 partners of P in Kp'
                const int c12 = same_n ? np : c1;         // d <= 2 partners (same 2M and parity keys)
                blen = (int64_t)(c12 - c1) + (int64_t)(c1 - d0) * bl1 + (int64_t)d0 * bl12;
                np = 0;
            }
        }
        if (MODE == kCount) {
            // only the row's own block (lane 0 of the first window) is walked
            // segment by segment: it is cut at the diagonal
            int64_t t = blen;
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
            pos += t;
        }
        const int bincl = wave_incl_scan(np);
        const int bstart = bincl - np;  // first segment of the lane's block
        const int S = lane63(bincl);
        int bcarry = -1;
        for (int s0 = 0; s0 < S; s0 += 64) {
            // 2. lane j: segment s0 + j = (target block, P'): its entry count
            const int s = s0 + lane;
            clear_marks(L);
            const int t = owner_of(L, bstart, np, s0, &bcarry);
            const int t_bp = lane_read(bp, t), t_start = lane_read(bstart, t);
            const int t_col = lane_read(bcol, t), t_str = lane_read(bstr, t);
            const int t_n1 = lane_read(bn1, t), t_l1 = lane_read(bl1, t);
            const int t_n12 = lane_read(bn12, t), t_l12 = lane_read(bl12, t);
            int len = 0;
            uint64_t pr = 0;
            int so = 0, sc = 0;
            if (s < S) {
                const int q = (t_bp & 0x7fffffff) + s - t_start;
                pr = t_bp < 0 ? P12[(uint32_t)q] : P1[(uint32_t)q];
                const int dp = rec_d(pr), ipp = rec_local(pr);
                sc = t_col + ipp * t_str;
                if (w0 + t == bi && ipp < ip && !R.full) {
                    len = 0;  // lower triangle
                } else if (dp == 2) {
                    len = 1;  // two protons moved: N' = N
                } else if (dp == 1) {
                    so = t_n1;
                    len = t_l1;
                } else {
                    so = t_n12 | (int)0x80000000;
                    len = t_l12;
                }
            }
            const int eincl = wave_incl_scan(len);
            const int T = lane63(eincl);
            if (MODE == kCount) {
                pos += T;
                continue;
            }
            const int estart = eincl - len;  // first entry of the lane's segment
            // 3. the entries of the chunk, 64 consecutive ones per round
            clear_marks(L);
            int ecarry = -1;
            // entries of this chunk of segments start at row position pos:
            // per-lane offsets from uniform bases stay 32-bit
            const int64_t base = R.pos0 + pos;
            const int room = (int)max((int64_t)0, min(R.cap - base, (int64_t)0x7fffffff));
            for (int e0 = 0; e0 < T; e0 += 64) {
                const int e = e0 + lane;
                const int j = owner_of(L, estart, len, e0, &ecarry);
                const uint64_t prj = lane_read64(pr, j);
                const int so2 = lane_read(so, j), sc2 = lane_read(sc, j), k = e - lane_read(estart, j);
                bool special = false;
                uint32_t qr = 0;
                if (e < T) {
                    const int dp = rec_d(prj);
                    uint64_t nr = 0;
                    if (dp != 2) {
                        const uint32_t idx = (uint32_t)((so2 & 0x7fffffff) + k);
                        nr = so2 < 0 ? N12[idx] : N1[idx];
                    }
                    const int dn = rec_d(nr);
                    special = (dp != 2) && (dp + dn != 2);
                    // two nucleons moved: pp (proton record), pn (both), nn (neutron record)
                    const int cls = dp == 2 ? 0 : (dp == 1 ? 1 : 2);
                    const int a = dp == 0 ? rec_p1(nr) : rec_p1(prj);
                    const int b = dp == 2 ? rec_p2(prj) : (dp == 1 ? rec_p1(nr) : rec_p2(nr));
                    const int c = dp == 0 ? rec_h1(nr) : rec_h1(prj);
                    const int d = dp == 2 ? rec_h2(prj) : (dp == 1 ? rec_h1(nr) : rec_h2(nr));
                    const bool neg = rec_neg(prj) ^ rec_neg(nr);
                    const bool inb = e < room;
                    const uint32_t ue = (uint32_t)e;
                    // upstream value first: its load overlaps the table lookup
                    const float gv = (MODE == kAdjoint && !special && inb) ? ld32(R.gval + base, ue) : 0.0f;
                    const int key = special ? -1 : tb_pos(B, cls, a, b, c, d);
                    if (inb) {
                        if (MODE == kFill) {
                            st32(R.col + base, ue, (int32_t)(sc2 + (dp == 2 ? in : rec_local(nr))));
                            if (!special) {
                                const float x = key >= 0 ? ld32(R.tbme, (uint32_t)key) : 0.0f;
                                st32(R.val + base, ue, neg ? -x : x);
                            }
                        } else if (key >= 0) {
                            adj_add(R, key, neg ? -gv : gv);
                        }
                    }
                    if (special) {
                        // queued: the moved nucleon's orbits and phase, or the diagonal
                        const uint64_t mr = dp == 1 ? prj : nr;
                        const uint32_t kind = dp == 1 ? 1u : (dn == 1 ? 2u : 0u);
                        qr = kind | ((uint32_t)rec_h1(mr) << 8) | ((uint32_t)rec_p1(mr) << 16) |
                             ((uint32_t)rec_neg(mr) << 24);
                    }
                    if (MODE == kFill && R.keys && inb)
                        st32(R.keys + base, ue, special ? (kKeySpecial | qr)
                                                        : (key >= 0 ? ((uint32_t)key | (neg ? kKeyNeg : 0u)) : kKeyNone));
                }
                if (MODE != kCount) {
                    // the diagonal entry (nothing moved) is treated on its own
                    const bool diag = special && q_kind(qr) == 0;
                    const uint64_t md = __ballot(diag);
                    if (md) diag_at = __builtin_amdgcn_readlane((int)(pos + e), __ffsll((long long)md) - 1);
                    special = special && !diag;
                }
                const uint64_t m = __ballot(special);
                if (m) {
                    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                    if (special) {
                        L.qpos[qn + rank] = (int32_t)(pos + e);
                        L.qrec[qn + rank] = qr;
                    }
                    qn += __popcll(m);
                    wave_sync();
                    if (qn > kQueue - 64) {  // room for one more round
                        flush_queue<MODE, true>(R, L, qn);
                        qn = 0;
                    }
                }
            }
            pos += T;
        }
    }
    if (MODE != kCount) flush_queue<MODE, true>(R, L, qn);
    if (MODE != kCount && diag_at >= 0) row_diagonal<MODE>(R, L, R.pos0 + diag_at);
    return pos;
}

// Adjoint of one row from the words the fill stored (R.keys): the row's
// entries [R.pos0, end) are read in order, single terms go straight to the
// accumulators and multi-term entries through the queue; the partner lists
// are not walked.
__device__ void do_row_keys(const BasisDev& B, WaveLds& L, int bi, int r, RowView& R, int64_t end)
{
    const int lane = threadIdx.x & 63;
    const int kp = uniform(cst(B.blk_kp)[bi]), kn = uniform(cst(B.blk_kn)[bi]);
    const cptr<int32_t> pkoff = cst(B.sp[0].key_off), nkoff = cst(B.sp[1].key_off);
    const int nKn = nkoff[kn + 1] - nkoff[kn];
    const int ip = uniform(r / nKn), in = uniform(r - ip * nKn);
    const int64_t n = (end < R.cap ? end : R.cap) - R.pos0;
    // software pipeline: the loads of the next 64 entries go out before the
    // current ones are accumulated (the first ones before the occupied orbits)
    uint32_t kn_ = 0;
    float gn_ = 0.0f;
    if (lane < n) {
        kn_ = glb(R.keys)[R.pos0 + lane];
        gn_ = glb(R.gval)[R.pos0 + lane];
    }
    row_occ(B, L, R, uniform(pkoff[kp] + ip), uniform(nkoff[kn] + in), false);
    int qn = 0;
    for (int64_t e0 = 0; e0 < n; e0 += 64) {
        const int64_t e = e0 + lane;
        const uint32_t k = kn_;
        const float g = gn_;
        if (e + 64 < n) {
            kn_ = glb(R.keys)[R.pos0 + e + 64];
            gn_ = glb(R.gval)[R.pos0 + e + 64];
        }
        const bool special = e < n && (k & kKeySpecial);
        if (e < n && !special && (k & kKeyPos) != kKeyNone) adj_add(R, (int)(k & kKeyPos), (k & kKeyNeg) ? -g : g);
        const uint64_t m = __ballot(special);
        if (m) {
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            if (special) {
                L.qpos[qn + rank] = (int32_t)e;
                L.qrec[qn + rank] = k & ~kKeySpecial;
            }
            qn += __popcll(m);
            wave_sync();
            if (qn > kQueue - 64) {  // room for one more round
                flush_queue<kAdjoint, false>(R, L, qn);
                qn = 0;
            }
        }
    }
    flush_queue<kAdjoint, false>(R, L, qn);
}

template <int MODE>
__device__ __forceinline__ void run_row_at(const BasisDev& B, int bi, int i, int r, const float* __restrict__ tbme,
                                           int64_t* __restrict__ row_ptr, int64_t nrp, int32_t* __restrict__ col,
                                           float* __restrict__ val, const float* __restrict__ gval,
                                           unsigned long long* __restrict__ gacc, lptr<uint32_t> hkey,
                                           lptr<int32_t> hval, bool use_table, int hbits, int qshift, bool full,
                                           uint32_t* keys, WaveLds& L);

// Row grow of the batch (rows of all bases are numbered consecutively) on the
// calling wavefront.
template <int MODE>
__device__ __forceinline__ void run_row(const BasisDev* __restrict__ bases, int nb,
                                        const int64_t* __restrict__ basis_row0, int64_t grow,
                                        const float* __restrict__ tbme, int64_t* __restrict__ row_ptr,
                                        int64_t nrp, int32_t* __restrict__ col, float* __restrict__ val,
                                        const float* __restrict__ gval, unsigned long long* __restrict__ gacc,
                                        lptr<uint32_t> hkey, lptr<int32_t> hval, bool use_table, bool full,
                                        uint32_t* keys, WaveLds& L)
{
    // basis of the row (few bases: linear search)
    int b = 0;
    while (b + 1 < nb && cst(basis_row0)[b + 1] <= grow) b++;
    b = uniform(b);
    const BasisDev& B = bases[b];
    const int i = uniform((int)(grow - cst(basis_row0)[b]));
    // block of the row
    const cptr<int64_t> blk_off = cst(B.blk_off);
    int lo = 0, hi = B.nblk;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (blk_off[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int bi = uniform(lo);
    run_row_at<MODE>(B, bi, i, i - (int)blk_off[bi], tbme, row_ptr, nrp, col, val, gval, gacc, hkey, hval, use_table,
                     0, 0, full, keys, L);
}

// Row i of basis B, row r of its block bi.
template <int MODE>
__device__ __forceinline__ void run_row_at(const BasisDev& B, int bi, int i, int r, const float* __restrict__ tbme,
                                           int64_t* __restrict__ row_ptr, int64_t nrp, int32_t* __restrict__ col,
                                           float* __restrict__ val, const float* __restrict__ gval,
                                           unsigned long long* __restrict__ gacc, lptr<uint32_t> hkey,
                                           lptr<int32_t> hval, bool use_table, int hbits, int qshift, bool full,
                                           uint32_t* keys, WaveLds& L)
{
    RowView R;
    R.B = &B;
    R.tbme = tbme ? tbme + B.tbme0 : nullptr;
    R.gacc = gacc ? gacc + B.tbme0 : nullptr;
    R.tbme0 = B.tbme0;
    R.hkey = hkey;
    R.hval = hval;
    R.use_table = use_table;
    R.hbits = hbits;
    R.qshift = qshift;
    R.gval = gval;
    R.col = col;
    R.val = val;
    R.keys = keys;
    R.Z = B.Z;
    R.NN = B.NN;
    R.spe_sum = 0.0;
    R.full = full;
    if (MODE == kCount) {
        R.pos0 = 0;
        R.cap = 0;
        const int64_t n = do_row<kCount>(B, L, bi, r, R);
        if ((threadIdx.x & 63) == 0) glbw(row_ptr)[B.row0 + i + 1] = n;
    } else {
        R.pos0 = uniform64(cst(row_ptr)[B.row0 + i]);
        R.cap = uniform64(cst(row_ptr)[nrp - 1]);  // the entries of all bases end here
        if (MODE == kAdjoint && keys)
            do_row_keys(B, L, bi, r, R, uniform64(cst(row_ptr)[B.row0 + i + 1]));
        else
            do_row<MODE>(B, L, bi, r, R);
    }
}

// Count and fill.  grab == 0: one wavefront per row over a grid of all rows.
// grab > 0: a persistent grid; each wavefront takes grab consecutive rows at a
// time from the work counter *queue (zero at launch) until none are left.
// Eight wavefronts per SIMD (the compiler keeps the fill within 64 VGPRs and
// spills a few registers): the fill is issue bound and the extra wavefront
// hides more of its load latency (10B fill 1.61 -> 1.54 ms, 6Li 0.64 -> 0.59).
template <int MODE, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(8, 8)))
    row_kernel(const BasisDev* __restrict__ bases, int nb, const int64_t* __restrict__ basis_row0,
               int64_t nrows, const float* __restrict__ tbme, int64_t* __restrict__ row_ptr, int64_t nrp,
               int32_t* __restrict__ col, float* __restrict__ val, uint32_t* __restrict__ keys, int grab,
               unsigned long long* __restrict__ queue, int full, int xcd)
{
    __shared__ WaveLds lds[WAVES];
    const int wid = uniform(threadIdx.x >> 6);
    if (grab <= 0) {
        const int64_t wg = xcd ? xcd_contiguous(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
        const int64_t grow = wg * WAVES + wid;
        if (grow < nrows)
            run_row<MODE>(bases, nb, basis_row0, grow, tbme, row_ptr, nrp, col, val, nullptr, nullptr, nullptr,
                          nullptr, false, full != 0, keys, lds[wid]);
        return;
    }
    for (;;) {
        unsigned long long t = 0;
        if ((threadIdx.x & 63) == 0)
            t = __hip_atomic_fetch_add(glbw(queue), (unsigned long long)grab, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        const int64_t g0 = uniform64((int64_t)t);
        if (g0 >= nrows) break;
        const int64_t g1 = g0 + grab < nrows ? g0 + grab : nrows;
        for (int64_t g = g0; g < g1; g++)
            run_row<MODE>(bases, nb, basis_row0, g, tbme, row_ptr, nrp, col, val, nullptr, nullptr, nullptr,
                          nullptr, false, full != 0, keys, lds[wid]);
    }
}

// Adjoint row groups: each block (proton key Kp, neutron key Kn) is cut into
// tiles of tp x tn determinants, tn = min(tile_n, |Kn|), tp = max(1, rows /
// tn); the rows of a tile share proton moves (same P) and neutron moves (same
// N), so their table positions repeat.  tile_off[gb + 1] (inclusive scan over
// the global block list of the batch) is the number of tiles of blocks <= gb.
__device__ __forceinline__ void block_tile_shape(int nKp, int nKn, int rows, int tile_n, int* tp, int* tn)
{
    const int n = tile_n < nKn ? tile_n : nKn;
    const int p = rows / n;
    *tn = n;
    *tp = p > 1 ? p : 1;
    (void)nKp;
}

__global__ void __launch_bounds__(256) tile_offsets(const BasisDev* __restrict__ bases,
                                                    const int32_t* __restrict__ blk_basis,
                                                    const int32_t* __restrict__ blk_local, int nblocks, int rows,
                                                    int tile_n, int64_t* __restrict__ tile_off, int nbases,
                                                    AdjBasis* __restrict__ adjb)
{
    __shared__ int64_t part[4];
    int64_t carry = 0;
    if (threadIdx.x == 0) tile_off[0] = 0;
    for (int g0 = 0; g0 < nblocks; g0 += 256) {
        const int gb = g0 + (int)threadIdx.x;
        int64_t n = 0;
        if (gb < nblocks) {
            const BasisDev& B = bases[blk_basis[gb]];
            const int bi = blk_local[gb];
            const int kn = B.blk_kn[bi];
            const int nKn = B.sp[1].key_off[kn + 1] - B.sp[1].key_off[kn];
            const int nKp = (int)((B.blk_off[bi + 1] - B.blk_off[bi]) / nKn);
            int tp, tn;
            block_tile_shape(nKp, nKn, rows, tile_n, &tp, &tn);
            n = (int64_t)((nKp + tp - 1) / tp) * ((nKn + tn - 1) / tn);
        }
        // inclusive scan over the 256 threads: wave scan, then wave totals
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        int64_t v = n;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t u = __shfl_up(v, o, 64);
            if (lane >= o) v += u;
        }
        if (lane == 63) part[w] = v;
        __syncthreads();
        int64_t add = carry;
        for (int k = 0; k < w; k++) add += part[k];
        if (gb < nblocks) tile_off[gb + 1] = v + add;
        carry += part[0] + part[1] + part[2] + part[3];
        __syncthreads();
    }
    // per-basis layout of the tile records: the blocks of a basis are
    // consecutive in the global block list, so are its tiles
    if (adjb && threadIdx.x == 0) {
        int blk0 = 0;
        int64_t hist0 = 0, bucket0 = 0;
        for (int x = 0; x < nbases; x++) {
            const BasisDev& B = bases[x];
            AdjBasis a;
            a.tile0 = tile_off[blk0];
            a.ntiles = tile_off[blk0 + B.nblk] - a.tile0;
            a.hist0 = hist0;
            a.bucket0 = bucket0;
            a.bits = adj_bucket_bits(B.ntbme);
            a.nb = adj_buckets(B.ntbme);
            adjb[x] = a;
            blk0 += B.nblk;
            hist0 += a.ntiles * (a.nb + 1);
            bucket0 += a.nb;
        }
    }
}

// Adjoint: a workgroup takes one tile of rows (above), its wavefronts take
// the tile's rows one at a time from a shared counter, and the contributions
// meet in the LDS accumulator table.  When the tile is done its occupied slots
// are written out as (table position, int32 fixed-point partial sum) records, grouped by
// bucket of the basis' table (a histogram row per tile gives each bucket's
// segment), with plain stores; adjoint_reduce sums them.  No device-scope
// atomic is issued except for a contribution that finds no slot within
// kAdjProbes probes (it goes to the int64 accumulator gacc directly).
// persistent == 0: tile = workgroup index; persistent == 1: a persistent grid
// takes tiles from the work counter *queue (zero at launch).  use_table == 0
// (global table positions do not fit 32 bits): every contribution goes to
// gacc and no record is written.
template <int WAVES, int SLOT_BITS>
__global__ void __launch_bounds__(64 * WAVES)
    adjoint_kernel(const BasisDev* __restrict__ bases, const int32_t* __restrict__ blk_basis,
                   const int32_t* __restrict__ blk_local, int nblocks, const int64_t* __restrict__ tile_off,
                   int rows, int tile_n, const int64_t* __restrict__ row_ptr, int64_t nrp,
                   const float* __restrict__ gval, const uint32_t* __restrict__ keys,
                   unsigned long long* __restrict__ gacc, int use_table, int persistent,
                   unsigned long long* __restrict__ queue, const AdjBasis* __restrict__ adjb,
                   uint64_t* __restrict__ recs, int64_t rec_cap, unsigned long long* __restrict__ rec_count,
                   int32_t* __restrict__ hist, const unsigned long long* __restrict__ gscale, int xcd)
{
    constexpr int kSlots = 1 << SLOT_BITS;
    constexpr int kThreads = 64 * WAVES;
    __shared__ WaveLds lds[WAVES];
    __shared__ uint32_t hkey[kSlots];
    __shared__ int32_t hval[kSlots];  // fixed-point tile sums
    __shared__ int32_t bcur[kAdjMaxBuckets + 1];  // bucket counts, then cursors
    __shared__ int next_row;
    __shared__ int t_gb, t_ip0, t_in0, t_tp, t_tn, t_nKn, t_valid;
    __shared__ int64_t t_g, t_base;
    for (int s = threadIdx.x; s < kSlots; s += kThreads) {
        hkey[s] = kAdjEmpty;
        hval[s] = 0;
    }
    const int wid = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t ntiles = tile_off[nblocks];
    for (;;) {
        if (threadIdx.x == 0) {
            next_row = 0;
            const int64_t g = persistent ? (int64_t)__hip_atomic_fetch_add(glbw(queue), 1ull, __ATOMIC_RELAXED,
                                                                            __HIP_MEMORY_SCOPE_AGENT)
                                         : (xcd ? xcd_contiguous(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x);
            t_valid = g < ntiles;
            t_g = g;
            if (g < ntiles) {
                // block of the tile: largest gb with tile_off[gb] <= g
                int lo = 0, hi = nblocks;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (tile_off[mid] <= g) lo = mid;
                    else hi = mid;
                }
                const BasisDev& B = bases[blk_basis[lo]];
                const int bi = blk_local[lo];
                const int kn = B.blk_kn[bi];
                const int nKn = B.sp[1].key_off[kn + 1] - B.sp[1].key_off[kn];
                const int nKp = (int)((B.blk_off[bi + 1] - B.blk_off[bi]) / nKn);
                int tp, tn;
                block_tile_shape(nKp, nKn, rows, tile_n, &tp, &tn);
                const int t = (int)(g - tile_off[lo]), ntn = (nKn + tn - 1) / tn;
                const int ip0 = (t / ntn) * tp, in0 = (t % ntn) * tn;
                t_gb = lo;
                t_ip0 = ip0;
                t_in0 = in0;
                t_tp = (nKp - ip0) < tp ? nKp - ip0 : tp;
                t_tn = (nKn - in0) < tn ? nKn - in0 : tn;
                t_nKn = nKn;
            }
        }
        __syncthreads();
        if (!t_valid) break;
        const int gb = uniform(t_gb), ip0 = uniform(t_ip0), in0 = uniform(t_in0), tp = uniform(t_tp),
                  tn = uniform(t_tn), nKn = uniform(t_nKn);
        const int64_t g = uniform64(t_g);
        const int xb = uniform(cst(blk_basis)[gb]);
        const BasisDev& B = bases[xb];
        const int bi = uniform(cst(blk_local)[gb]);
        const int cnt = tp * tn;
        const int qshift = uniform((int)(int64_t)cst(gscale)[xb]);
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&next_row, 1);
            t = uniform(t);
            if (t >= cnt) break;
            const int u = t / tn, v = t - u * tn;
            const int r = (ip0 + u) * nKn + in0 + v;
            run_row_at<kAdjoint>(B, bi, uniform((int)cst(B.blk_off)[bi] + r), r, nullptr, const_cast<int64_t*>(row_ptr), nrp,
                                 nullptr, nullptr, gval, gacc, (lptr<uint32_t>)hkey, (lptr<int32_t>)hval,
                                 use_table != 0, SLOT_BITS, qshift, false, const_cast<uint32_t*>(keys), lds[wid]);
        }
        __syncthreads();
        if (use_table) {
            // records of the tile, grouped by bucket: count, reserve room in
            // the record buffer (one device-scope atomic per tile), scan (one
            // wavefront; the histogram row of absolute positions goes to
            // global memory), scatter.  Without room (or without a record
            // buffer) the slots go to the int64 accumulators instead.
            const AdjBasis A = adjb ? adjb[xb] : AdjBasis{};
            const uint32_t base = (uint32_t)B.tbme0;
            if (recs) {
                for (int i = threadIdx.x; i <= A.nb; i += kThreads) bcur[i] = 0;
                __syncthreads();
                for (int s = threadIdx.x; s < kSlots; s += kThreads) {
                    const uint32_t k = hkey[s];
                    if (k != kAdjEmpty) atomicAdd(&bcur[(k - base) >> A.bits], 1);
                }
                __syncthreads();
                if (wid == 0) {
                    int run = 0;
                    for (int c0 = 0; c0 < A.nb; c0 += 64) {
                        const int c = c0 + lane;
                        const int v = c < A.nb ? bcur[c] : 0;
                        const int incl = wave_incl_scan(v);
                        if (c < A.nb) bcur[c] = run + incl - v;
                        run += lane63(incl);
                    }
                    if (lane == 0) {
                        int64_t at = (int64_t)__hip_atomic_fetch_add(glbw(rec_count), (unsigned long long)run,
                                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (at + run > rec_cap) at = -1;
                        t_base = at;
                        bcur[A.nb] = run;
                    }
                }
                __syncthreads();
                const int64_t at = t_base;
                // column g - tile0 of the basis' histogram, bucket-major (the
                // reduction reads one bucket's row of every tile contiguously)
                const gmut<int32_t> hcol = glbw(hist) + A.hist0 + (g - A.tile0);
                for (int c = threadIdx.x; c <= A.nb; c += kThreads)
                    hcol[(int64_t)c * A.ntiles] = at >= 0 ? (int32_t)(at + bcur[c]) : 0;
                __syncthreads();
                if (at >= 0) {
                    const gmut<uint64_t> out = glbw(recs) + at;
                    for (int s = threadIdx.x; s < kSlots; s += kThreads) {
                        const uint32_t k = hkey[s];
                        if (k != kAdjEmpty) {
                            const int p = atomicAdd(&bcur[(k - base) >> A.bits], 1);
                            out[p] = (uint64_t)k | ((uint64_t)(uint32_t)hval[s] << 32);
                            hkey[s] = kAdjEmpty;
                            hval[s] = 0;
                        }
                    }
                }
            }
            for (int s = threadIdx.x; s < kSlots; s += kThreads) {
                const uint32_t k = hkey[s];
                if (k != kAdjEmpty) {  // no record buffer, or no room in it
                    atomic_add_i64(glbw(gacc) + k, (int64_t)hval[s]);
                    hkey[s] = kAdjEmpty;
                    hval[s] = 0;
                }
            }
        }
        __syncthreads();
        if (!persistent) break;
    }
}

// Sum of the adjoint's tile records.  hist holds, per basis, nb + 1 rows of
// one int32 per tile: row j, the absolute record position where the tile's
// records of bucket j start (row nb: where its last bucket ends).  Workgroup (bucket, c) sums the bucket's records of the c-th of
// `chunks` equal slices of the basis' tiles: each wavefront takes 64 tiles at a
// time (lane l: tile t0 + l, its segment of the bucket) and every lane walks
// its own segment, four records per step; the sums meet in an int64
// shared-memory array of up to 2^kAdjReduceBits positions (a larger bucket is
// summed window by window).  With one chunk the workgroup adds the direct
// contributions in gacc and writes each position once as FP32; with several it
// writes its int64 partial sums to part[c] and adjoint_combine adds the chunks.
constexpr int kReduceThreads = 256;
constexpr int kReduceWindow = 1 << kAdjReduceBits;

__global__ void __launch_bounds__(kReduceThreads)
    adjoint_reduce(const BasisDev* __restrict__ bases, const AdjBasis* __restrict__ adjb, int nbases,
                   const uint64_t* __restrict__ recs, const int32_t* __restrict__ hist,
                   const unsigned long long* __restrict__ gacc, float* __restrict__ gtbme, int chunks,
                   unsigned long long* __restrict__ part, int64_t ntbme_all,
                   const unsigned long long* __restrict__ gscale)
{
    __shared__ unsigned long long acc[kReduceWindow];
    const int64_t bucket = blockIdx.x / chunks;
    const int c = (int)(blockIdx.x - bucket * chunks);
    // basis of the bucket: largest x with bucket0 <= bucket
    int lo = 0, hi = nbases;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (adjb[mid].bucket0 <= bucket) lo = mid;
        else hi = mid;
    }
    const int x = uniform(lo);
    const int qshift = (int)(int64_t)gscale[x];
    const AdjBasis A = adjb[x];
    const int64_t tbme0 = bases[x].tbme0, ntbme = bases[x].ntbme;
    const int j = (int)(bucket - A.bucket0);
    const int64_t klo = (int64_t)j << A.bits;
    const int64_t khi = (klo + ((int64_t)1 << A.bits)) < ntbme ? klo + ((int64_t)1 << A.bits) : ntbme;
    const int64_t ta = A.ntiles * c / chunks, tb = A.ntiles * (c + 1) / chunks;  // this chunk's tiles
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    constexpr int kWaves = kReduceThreads / 64;
    for (int64_t w0 = klo; w0 < khi; w0 += kReduceWindow) {
        const int64_t w1 = (w0 + kReduceWindow) < khi ? w0 + kReduceWindow : khi;
        const int wn = (int)(w1 - w0);
        for (int i = threadIdx.x; i < wn; i += kReduceThreads) acc[i] = 0;
        __syncthreads();
        const int64_t kb = tbme0 + w0;  // global table position of acc[0]
        for (int64_t t0 = ta + (int64_t)wid * 64; t0 < tb; t0 += (int64_t)kWaves * 64) {
            const int64_t t = t0 + lane;
            int64_t p = 0, e = 0;
            if (t < tb) {
                const gptr<int32_t> hr = glb(hist) + A.hist0 + t;
                p = hr[(int64_t)j * A.ntiles];
                e = hr[(int64_t)(j + 1) * A.ntiles];
            }
            for (; p + 4 <= e; p += 4) {
                uint64_t r[4];
#pragma unroll
                for (int u = 0; u < 4; u++) r[u] = glb(recs)[p + u];
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const int64_t k = (int64_t)(uint32_t)r[u] - kb;
                    if (k >= 0 && k < wn) atomicAdd(&acc[k], (unsigned long long)(int64_t)(int32_t)(r[u] >> 32));
                }
            }
            for (; p < e; p++) {
                const uint64_t r = glb(recs)[p];
                const int64_t k = (int64_t)(uint32_t)r - kb;
                if (k >= 0 && k < wn) atomicAdd(&acc[k], (unsigned long long)(int64_t)(int32_t)(r >> 32));
            }
        }
        __syncthreads();
        if (chunks == 1) {
            for (int i = threadIdx.x; i < wn; i += kReduceThreads)
                gtbme[kb + i] = fixed_to_f32(acc[i] + gacc[kb + i], qshift);
        } else {
            for (int i = threadIdx.x; i < wn; i += kReduceThreads) part[(int64_t)c * ntbme_all + kb + i] = acc[i];
        }
        __syncthreads();
    }
}

// fixed-point shift of table position k of the batch (bases in table order)
__device__ __forceinline__ int shift_of(const BasisDev* __restrict__ bases, int nbases,
                                        const unsigned long long* __restrict__ gscale, int64_t k)
{
    int lo = 0, hi = nbases;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bases[mid].tbme0 <= k) lo = mid;
        else hi = mid;
    }
    return (int)(int64_t)gscale[lo];
}

// gtbme = gacc + the chunks' partial sums
__global__ void __launch_bounds__(256) adjoint_combine(const unsigned long long* __restrict__ gacc,
                                                       const unsigned long long* __restrict__ part, int chunks,
                                                       int64_t n, float* __restrict__ gtbme,
                                                       const BasisDev* __restrict__ bases, int nbases,
                                                       const unsigned long long* __restrict__ gscale)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        unsigned long long v = gacc[k];
        for (int c = 0; c < chunks; c++) v += part[(int64_t)c * n + k];
        gtbme[k] = fixed_to_f32(v, shift_of(bases, nbases, gscale, k));
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

__global__ void fixed_to_f32_n(const unsigned long long* __restrict__ x, float* __restrict__ y, int64_t n,
                               const BasisDev* __restrict__ bases, int nbases,
                               const unsigned long long* __restrict__ gscale)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        y[t] = fixed_to_f32(x[t], shift_of(bases, nbases, gscale, t));
}

// max |G| of each basis over its stored entries, as the bits of a
// non-negative FP32 (ordered like the values), into gscale[basis] (zero
// before).  The entries of the batch (bases in row order hold consecutive
// entry ranges) are cut into chunks of `chunk` entries (a multiple of 4);
// workgroup c takes chunks c, c + gridDim.x, ... and reduces each basis a chunk
// overlaps (nearly always one), so large and small bases get workgroups in
// proportion to their entries.
constexpr int kAbsThreads = 256;

__device__ __forceinline__ uint32_t absmax_range(const float* __restrict__ g, int64_t n0, int64_t n1)
{
    // 16-byte loads over the 16-byte aligned middle [a0, a1) of the range
    const int64_t a0 = min(n1, n0 + (int64_t)(((16 - ((uintptr_t)(g + n0) & 15)) & 15) / 4));
    const int64_t a1 = a0 + ((n1 - a0) & ~(int64_t)3);
    uint32_t m = 0;
    const float4* v = (const float4*)(g + a0);
    for (int64_t t = threadIdx.x; t < (a1 - a0) / 4; t += kAbsThreads) {
        const float4 x = v[t];
        m = max(m, max(max(__float_as_uint(x.x) & 0x7fffffffu, __float_as_uint(x.y) & 0x7fffffffu),
                       max(__float_as_uint(x.z) & 0x7fffffffu, __float_as_uint(x.w) & 0x7fffffffu)));
    }
    for (int64_t t = n0 + threadIdx.x; t < a0; t += kAbsThreads) m = max(m, __float_as_uint(g[t]) & 0x7fffffffu);
    for (int64_t t = a1 + threadIdx.x; t < n1; t += kAbsThreads) m = max(m, __float_as_uint(g[t]) & 0x7fffffffu);
    return m;
}

__global__ void __launch_bounds__(kAbsThreads) grad_absmax(const float* __restrict__ g,
                                                           const int64_t* __restrict__ row_ptr,
                                                           const BasisDev* __restrict__ bases, int nbases,
                                                           int64_t chunk, unsigned long long* __restrict__ gscale)
{
    __shared__ uint32_t wmax[kAbsThreads / 64];
    const int64_t n = row_ptr[bases[nbases - 1].row0 + bases[nbases - 1].dim];  // entries of all bases
    for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < n; c0 += (int64_t)gridDim.x * chunk) {
        const int64_t c1 = min(c0 + chunk, n);
        // the basis whose entries hold c0
        int lo = 0, hi = nbases;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (row_ptr[bases[mid].row0] <= c0) lo = mid;
            else hi = mid;
        }
        for (int b = lo; b < nbases; b++) {
            const int64_t s0 = max(c0, row_ptr[bases[b].row0]);
            const int64_t s1 = min(c1, row_ptr[bases[b].row0 + bases[b].dim]);
            if (s0 >= c1) break;
            uint32_t m = s0 < s1 ? absmax_range(g, s0, s1) : 0u;
            for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
            if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t w = 0;
                for (int k = 0; k < kAbsThreads / 64; k++) w = max(w, wmax[k]);
                if (w) atomicMax(gscale + b, (unsigned long long)w);
            }
            __syncthreads();
        }
    }
}

// max |G| of each basis -> its fixed-point shift: with max |G| < 2^e and tiles
// of at most 2^rows_log2 rows, a contribution rounds to an integer of
// magnitude at most 2^(30 - rows_log2) and a tile's sum in one LDS slot stays
// below 2^30.  A zero (or non-finite) maximum gives shift 0.
__global__ void __launch_bounds__(256) adj_scale(unsigned long long* __restrict__ gscale, int nbases, int rows_log2)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbases) return;
    const float m = __uint_as_float((uint32_t)gscale[b]);
    int e = 0;
    (void)frexpf(m, &e);  // m = f * 2^e, 0.5 <= f < 1
    const int shift = (m > 0.0f && isfinite(m)) ? 30 - rows_log2 - e : 0;
    gscale[b] = (unsigned long long)(int64_t)shift;
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

__global__ void zero_u64(unsigned long long* __restrict__ p) { *p = 0; }

// Workgroups of a persistent grid: as many as the device holds at once.
// kind numbers the kernel for the per-device cache.
static unsigned resident_blocks(const void* kernel, int threads, int kind)
{
    constexpr int kDevs = 64, kKinds = 8;
    static std::atomic<int> cache[kDevs][kKinds];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevs) dev = 0;
    int v = cache[dev][kind].load(std::memory_order_relaxed);
    if (v <= 0) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per <= 0)
            per = 1;
        v = cus * per;
        cache[dev][kind].store(v, std::memory_order_relaxed);
    }
    return (unsigned)v;
}

template <int MODE, int WAVES>
static void launch_rows_w(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                          const float* tbme, int64_t* row_ptr, int64_t nrp, int32_t* col, float* val, uint32_t* keys,
                          int grab, unsigned long long* queue, int full, int xcd, hipStream_t s)
{
    unsigned grid = grid_for(nrows, WAVES);
    if (grab > 0) {
        hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, queue);
        const unsigned res = resident_blocks((const void*)row_kernel<MODE, WAVES>, 64 * WAVES,
                                             2 * MODE + (WAVES == 8 ? 1 : 0));
        const unsigned need = grid_for(nrows, WAVES * grab);
        grid = res < need ? res : need;
    }
    hipLaunchKernelGGL((row_kernel<MODE, WAVES>), dim3(grid), dim3(64 * WAVES), 0, s, bases, nb, basis_row0,
                       nrows, tbme, row_ptr, nrp, col, val, keys, grab, queue, full, xcd);
}

template <int MODE>
static hipError_t launch_rows(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                              const float* tbme, int64_t* row_ptr, int64_t nrp, int32_t* col, float* val,
                              uint32_t* keys, const ci_tuning& t, unsigned long long* queue, int full, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    if (t.row_waves == 8)
        launch_rows_w<MODE, 8>(bases, nb, basis_row0, nrows, tbme, row_ptr, nrp, col, val, keys, t.row_grab, queue,
                               full, t.row_xcd, s);
    else
        launch_rows_w<MODE, 4>(bases, nb, basis_row0, nrows, tbme, row_ptr, nrp, col, val, keys, t.row_grab, queue,
                               full, t.row_xcd, s);
    return hipGetLastError();
}

hipError_t launch_count(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                        int64_t* row_ptr, int64_t nrp, const int64_t* seg_first, int64_t* scan_tmp,
                        const ci_tuning& t, unsigned long long* queue, int full, hipStream_t s)
{
    hipError_t e = launch_rows<kCount>(bases, nb, basis_row0, nrows, nullptr, row_ptr, nrp, nullptr, nullptr,
                                       nullptr, t, queue, full, s);
    if (e != hipSuccess) return e;
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
                       uint32_t* keys, const ci_tuning& t, unsigned long long* queue, int full, hipStream_t s)
{
    return launch_rows<kFill>(bases, nb, basis_row0, nrows, tbme, const_cast<int64_t*>(row_ptr), nrp, col, val, keys,
                              t, queue, full, s);
}

hipError_t launch_vjp(const BasisDev* bases, int nbases, const int32_t* blk_basis, const int32_t* blk_local,
                      int nblocks, int64_t ntiles, int64_t* tile_off, AdjBasis* adjb, int64_t nbuckets, int chunks,
                      unsigned long long* part,
                      int64_t nrows, const int64_t* row_ptr, int64_t nrp, const float* gval, const uint32_t* keys,
                      float* gtbme, unsigned long long* gacc, uint64_t* recs, int64_t rec_cap,
                      unsigned long long* rec_count, int32_t* hist, int64_t ntbme, const ci_tuning& t,
                      unsigned long long* queue, unsigned long long* gscale, int64_t nnz_total, hipStream_t s)
{
    const unsigned gz = grid_for(ntbme, 256) < 4096 ? grid_for(ntbme, 256) : 4096;
    if (ntbme > 0) hipLaunchKernelGGL(fill_f64, dim3(gz), dim3(256), 0, s, (double*)gacc, ntbme, 0.0);  // int64 zeros
    const int use_table = ntbme < (int64_t)kAdjEmpty ? 1 : 0;
    const bool walked = nrows > 0 && ntiles > 0;
    const int rows = keys ? t.adjk_rows : t.adj_rows, tile_n = keys ? t.adjk_tile_n : t.adj_tile_n;
    // fixed-point shift from max |G| and the rows of a tile (at most max(rows, tile_n))
    int rows_log2 = 0;
    while ((1 << rows_log2) < (rows > tile_n ? rows : tile_n)) rows_log2++;
    if (nbases <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64, dim3(1), dim3(256), 0, s, (double*)gscale, (int64_t)nbases, 0.0);  // zeros
    if (nrows > 0) {
        // about 2048 workgroups (a few per CU, each streaming a long chunk) once
        // the host knows the entries (after the count); chunks of 16Ki..1Mi entries
        const int64_t chunk =
            nnz_total >= 0 ? std::min<int64_t>((int64_t)1 << 20, std::max<int64_t>(16384, (nnz_total / 2048 + 3) & ~(int64_t)3))
                           : 16384;
        const int64_t ch = nnz_total >= 0 ? (nnz_total + chunk - 1) / chunk : 4096;
        const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ch, (int64_t)1 << 20));
        hipLaunchKernelGGL(grad_absmax, dim3(grid), dim3(kAbsThreads), 0, s, gval, row_ptr, bases, nbases, chunk,
                           gscale);
    }
    hipLaunchKernelGGL(adj_scale, dim3(grid_for(nbases, 256)), dim3(256), 0, s, gscale, nbases, rows_log2);
    if (walked) {
        hipLaunchKernelGGL(tile_offsets, dim3(1), dim3(256), 0, s, bases, blk_basis, blk_local, nblocks, rows, tile_n,
                           tile_off, nbases, adjb);
        const bool wide = keys || t.adj_wide;  // 16 wavefronts, 16384-slot table
        const void* kern = wide ? (const void*)adjoint_kernel<kAdjKeysWaves, kAdjKeysSlotBits>
                                : (const void*)adjoint_kernel<kAdjWaves, kAdjSlotBits>;
        const int threads = 64 * (wide ? kAdjKeysWaves : kAdjWaves);
        unsigned grid = (unsigned)ntiles;
        if (recs) hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, rec_count);
        if (t.adj_persistent) {
            hipLaunchKernelGGL(zero_u64, dim3(1), dim3(1), 0, s, queue);
            const unsigned res = resident_blocks(kern, threads, wide ? 7 : 6);
            grid = res < grid ? res : grid;
        }
        if (wide)
            hipLaunchKernelGGL((adjoint_kernel<kAdjKeysWaves, kAdjKeysSlotBits>), dim3(grid), dim3(threads), 0, s,
                               bases, blk_basis, blk_local, nblocks, tile_off, rows, tile_n, row_ptr, nrp, gval, keys,
                               gacc, use_table, t.adj_persistent ? 1 : 0, queue, adjb, recs, rec_cap, rec_count,
                               hist, gscale, t.row_xcd);
        else
            hipLaunchKernelGGL((adjoint_kernel<kAdjWaves, kAdjSlotBits>), dim3(grid), dim3(threads), 0, s, bases,
                               blk_basis, blk_local, nblocks, tile_off, rows, tile_n, row_ptr, nrp, gval, keys, gacc,
                               use_table, t.adj_persistent ? 1 : 0, queue, adjb, recs, rec_cap, rec_count, hist,
                               gscale, t.row_xcd);
    }
    if (ntbme > 0) {
        if (use_table && walked && recs && nbuckets > 0) {
            const int ch = (chunks > 1 && part) ? chunks : 1;
            hipLaunchKernelGGL(adjoint_reduce, dim3((unsigned)(nbuckets * ch)), dim3(kReduceThreads), 0, s, bases,
                               adjb, nbases, recs, hist, gacc, gtbme, ch, part, ntbme, gscale);
            if (ch > 1)
                hipLaunchKernelGGL(adjoint_combine, dim3(gz), dim3(256), 0, s, gacc, part, ch, ntbme, gtbme, bases,
                                   nbases, gscale);
        } else
            hipLaunchKernelGGL(fixed_to_f32_n, dim3(gz), dim3(256), 0, s, gacc, gtbme, ntbme, bases, nbases, gscale);
    }
    return hipGetLastError();
}

// Slots of the shared-memory table of each adjoint (the records a tile can write).
int adjoint_slots(bool wide) { return wide ? (1 << kAdjKeysSlotBits) : (1 << kAdjSlotBits); }

}  // namespace ci
