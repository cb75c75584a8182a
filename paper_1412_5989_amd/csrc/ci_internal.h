// Internal definitions shared by the host index builder, the C ABI and the
// HIP kernels of libci.  Not part of the public interface (include/ci.h).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "ci.h"

#ifdef __HIPCC__
#define CI_HD __host__ __device__
#else
#define CI_HD
#endif

namespace ci {

constexpr int kMaxWords = 4;   // n_sps <= 256 per species

// ---------------------------------------------------------------------------
// Partner record of a species determinant x: one y with d(x, y) <= 2, where
// d is the number of orbits occupied in x and not in y.  Row-side orbits
// ("particles", in x not y) are p1 < p2; column-side orbits ("holes", in y not
// x) are h1 < h2.  The sign is the species-local fermion phase of the
// Slater-Condon element <x..|H|y..> (one- and two-nucleon moves).
//   bits  0..23  local index of y inside its species key
//   bits 24..31  h1    bits 32..39  p1    bits 40..47  h2    bits 48..55  p2
//   bit  56      phase is -1
//   bits 57..58  d (0, 1, 2)
// ---------------------------------------------------------------------------
constexpr uint64_t kRecLocalMask = (1ull << 24) - 1;

CI_HD inline uint64_t make_rec(uint32_t ylocal, int d, int h1, int p1, int h2, int p2, bool neg)
{
    return (uint64_t)ylocal | ((uint64_t)(h1 & 255) << 24) | ((uint64_t)(p1 & 255) << 32) |
           ((uint64_t)(h2 & 255) << 40) | ((uint64_t)(p2 & 255) << 48) |
           ((uint64_t)(neg ? 1 : 0) << 56) | ((uint64_t)d << 57);
}

// two-body pair index entry (host): (sector << 16) | position of the pair in the sector
constexpr uint32_t kNoPair = 0xffffffffu;
// device pair entry: bits 0..15 position r of the pair in its sector, bits
// 16..31 sector, bits 32..63 base(r) = sector offset + r (2 n_s - r + 1) / 2 - r,
// so that V_{r,q} (r <= q) sits at base(r) + q
constexpr uint64_t kNoPair64 = ~0ull;

// ---------------------------------------------------------------------------
// Device view of one species (all pointers into the basis arena).
// ---------------------------------------------------------------------------
struct SpeciesDev {
    const uint64_t* sd;      // [nsd][W]
    const int32_t* key_off;  // [nk + 1] first global index of each key
    const int64_t* l1_ptr;   // [nsd + 1] start of the d<=1 list of x
    const int64_t* l12_ptr;  // [nsd + 1] start of the d<=2 list of x
    const uint64_t* l1;      // d<=1 partners (self included), all keys, y ascending
    const uint64_t* l12;     // d<=2 partners in keys of the same 2M and Nq parity
    const int32_t* seg1;     // [nsd][nk + 1] first record of each key in l1(x)
    const int32_t* seg12;    // [nsd][nk + 1] same for l12(x)
    const int32_t* self12;   // [nsd] position of x itself inside its own key segment of l12(x)
    int32_t nsd, nk;
};

// One block (proton key, neutron key) as one 16-byte record.
struct alignas(16) BlockInfo {
    int32_t kp, kn;  // proton and neutron key
    int32_t row0;    // first row (the block offset)
    int32_t nkn;     // rows per proton determinant (|Kn|)
};

struct BasisDev {
    SpeciesDev sp[2];          // 0 = protons, 1 = neutrons
    const BlockInfo* blk;      // [nblk]
    const int32_t* blk_kp;     // [nblk]
    const int32_t* blk_kn;     // [nblk]
    const int64_t* blk_off;    // [nblk + 1] first row of each block
    const uint64_t* pair;      // [3][n][n] pp, pn, nn pair entries (species-local orbits)
    const int32_t* orb_n;      // [n] oscillator shell of each orbit
    const int32_t* orb_qn;     // [n] n | l << 8 | 2j << 16 | (2m + 64) << 24 of each orbit
    int64_t dim;               // D
    int64_t row0;              // R_b: this basis' segment of row_ptr
    int64_t tbme0;             // T_b: this basis' slice of the two-body table
    int64_t ntbme;             // length of this basis' table
    int32_t W, nsps, nblk, nsec, Z, NN;
    int32_t kinetic;           // off-diagonal oscillator kinetic term in the one-body part
    double hw;
};


// Adjoint: the table positions of one basis are cut into buckets of 2^bits
// consecutive positions (bits >= kAdjBucketMinBits, chosen so that a basis has
// at most kAdjMaxBuckets buckets).  Every adjoint tile writes the partial sums
// of its shared-memory table as (position, value) records grouped by bucket,
// and a histogram row of nb + 1 offsets; one workgroup per bucket then sums
// the records of every tile of its basis.  Per basis, for one launch shape
// (tile_offsets computes it on the device, the host the same sizes):
struct AdjBasis {
    int64_t tile0;    // first tile of the basis (global tile index)
    int64_t ntiles;   // tiles of the basis
    int64_t hist0;    // first histogram entry of the basis (ntiles rows of nb + 1)
    int64_t bucket0;  // first bucket of the basis (global bucket index)
    int32_t nb;       // buckets of the basis
    int32_t bits;     // log2 of the positions per bucket
};
constexpr int kAdjBucketMinBits = 13;  // at least 2^13 positions per bucket
constexpr int kAdjMaxBuckets = 1024;
constexpr int kAdjReduceBits = 13;     // the reducing workgroup sums 2^13 positions at a time
constexpr int kAdjMaxChunks = 16;      // tile chunks per bucket in the reduction

CI_HD inline int adj_bucket_bits(int64_t ntbme)
{
    int bits = kAdjBucketMinBits;
    while (((ntbme + ((int64_t)1 << bits) - 1) >> bits) > kAdjMaxBuckets) bits++;
    return bits;
}
CI_HD inline int adj_buckets(int64_t ntbme)
{
    const int bits = adj_bucket_bits(ntbme);
    return (int)((ntbme + ((int64_t)1 << bits) - 1) >> bits);
}

// ---------------------------------------------------------------------------
// Host-side tables of one basis.
// ---------------------------------------------------------------------------
struct HostSpecies {
    int X = 0;                      // particles
    int budget = 0;                 // largest Nq of one determinant
    std::vector<int32_t> key_nq, key_m2;
    std::vector<int32_t> key_off;   // nk + 1
    std::vector<uint64_t> sd;       // nsd * W
    std::vector<int32_t> sd_key;    // nsd
    int nk() const { return (int)key_nq.size(); }
    int64_t nsd() const { return (int64_t)sd_key.size(); }
};

struct HostBasis {
    ci_problem prob{};
    int S = 0, nsps = 0, W = 0, N0 = 0, N0p = 0, N0n = 0;
    std::vector<int32_t> orb_n, orb_l, orb_j2, orb_m2;  // species-local orbits
    HostSpecies sp[2];
    std::vector<int32_t> blk_kp, blk_kn;
    std::vector<int64_t> blk_off;
    int64_t dim = 0;
    std::vector<int64_t> sec_off;
    std::vector<int32_t> sec_n;
    std::vector<uint32_t> pair;    // 3 * n * n: sector << 16 | position, or kNoPair
    int64_t n_tbme = 0;
    int nblk() const { return (int)blk_kp.size(); }
};

// Arguments of the device partner-list kernels (basis_kernels.hip), one species.
struct PartnerArgs {
    const uint64_t* sd;      // [nsd][W]
    const uint64_t* sdT;     // [W][nsd] (word-major copy for coalesced candidate loads)
    const int32_t* sd_key;   // [nsd]
    const int32_t* key_off;  // [nk + 1]
    const int32_t* key_nq;   // [nk]
    const int32_t* key_m2;   // [nk]
    int64_t* l1_ptr;         // count pass: counts at [x + 1]; fill pass: offsets
    int64_t* l12_ptr;
    uint64_t* l1;
    uint64_t* l12;
    int32_t* seg1;  // [nsd][nk + 1]
    int32_t* seg12;
    int32_t* self12;
    int32_t nsd, nk, W;
};

// host_basis.cpp
int validate_problem(const ci_problem& p, std::string& err);
// Host tables: orbits, species determinants, keys, blocks, table sectors and
// pair index (the partner lists are built on the device).
int plan_basis(const ci_problem& p, HostBasis& hb, std::string& err);
// The same in parts: the orbits (validates the problem first); the
// determinants, keys and blocks (needs the orbits); the two-body sectors and
// pair index (needs only the orbits, so it can run on another thread while
// the determinants are enumerated: the two parts write disjoint members).
int plan_orbits(const ci_problem& p, HostBasis& hb, std::string& err);
int plan_determinants(HostBasis& hb, std::string& err);
int plan_tbme_index(HostBasis& hb, std::string& err);
// Two-body keys (a, b, c, d) in table order.
void tbme_keys(const HostBasis& hb, std::vector<int32_t>& abcd);
// Device form of the pair index ([3][n][n] uint64: base of the pair row << 32 | sector << 16 | position).
void write_pair64(const HostBasis& hb, uint64_t* out);

}  // namespace ci
