// Host construction of the basis indexing of one problem (paper Sec. 2: the
// indexing systems of the many-body basis are set up before the matrix is
// built; Sec. 5.2: index structures are built contiguously on the host and
// moved to the device with one allocation and one copy).
//
// Builds: the oscillator orbits; the proton and neutron determinants grouped
// by (Nq, 2M) key; the compatible key blocks and row offsets; for every
// species determinant its one- and two-nucleon partner lists with the moved
// orbits and the fermion phase; the sector / pair index of the two-body table;
// all flat, for a single upload.
#include <algorithm>
#include <array>
#include <cstring>
#include <functional>
#include <map>
#include <thread>
#include <unordered_map>

#include "ci_internal.h"

namespace ci {

namespace {

int shell_capacity(int N) { return (N + 1) * (N + 2); }

// shell of the X-th nucleon when shells fill from the bottom
int top_shell(int X)
{
    int N = 0, filled = 0;
    if (X <= 0) return 0;
    while (filled + shell_capacity(N) < X) filled += shell_capacity(N++);
    return N;
}

// total oscillator quanta of the lowest filling of X nucleons
int lowest_quanta(int X)
{
    int s = 0;
    for (int N = 0, left = X; left > 0; N++) {
        int take = std::min(left, shell_capacity(N));
        s += take * N;
        left -= take;
    }
    return s;
}

using Bits = std::array<uint64_t, kMaxWords>;

struct BitsHash {
    size_t operator()(const Bits& b) const
    {
        uint64_t h = 0x9e3779b97f4a7c15ull;
        for (uint64_t w : b) {
            uint64_t z = w + h;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            h = z ^ (z >> 31);
        }
        return (size_t)h;
    }
};

inline bool test_bit(const Bits& b, int k) { return (b[k >> 6] >> (k & 63)) & 1; }
inline void flip_bit(Bits& b, int k) { b[k >> 6] ^= 1ull << (k & 63); }

// number of set bits of b strictly below orbit k
inline int count_below(const Bits& b, int k)
{
    int c = 0;
    for (int w = 0; w < (k >> 6); w++) c += __builtin_popcountll(b[w]);
    if (k & 63) c += __builtin_popcountll(b[k >> 6] & ((1ull << (k & 63)) - 1));
    return c;
}

struct RawSD {
    Bits bits;
    int nq, m2;
};

void enumerate_species(const HostBasis& hb, int X, int budget, std::vector<RawSD>& out)
{
    const int n = hb.nsps;
    RawSD cur{};
    // depth-first choice of X orbits in ascending order
    std::function<void(int, int, int, int)> rec = [&](int start, int left, int nq, int m2) {
        if (left == 0) {
            cur.nq = nq;
            cur.m2 = m2;
            out.push_back(cur);
            return;
        }
        for (int k = start; k <= n - left; k++) {
            // orbits ascend in N, so the remaining picks cost at least left * N_k
            if (nq + left * hb.orb_n[k] > budget) break;
            flip_bit(cur.bits, k);
            rec(k + 1, left - 1, nq + hb.orb_n[k], m2 + hb.orb_m2[k]);
            flip_bit(cur.bits, k);
        }
    };
    rec(0, X, 0, 0);
}

bool colex_less(const uint64_t* a, const uint64_t* b, int W)
{
    for (int w = W - 1; w >= 0; w--)
        if (a[w] != b[w]) return a[w] < b[w];
    return false;
}

bool block_ok(const HostBasis& hb, int nqp, int m2p, int nqn, int m2n)
{
    int nq = nqp + nqn;
    if (nq > hb.N0 + hb.prob.nmax) return false;
    if (((nq & 1) ? -1 : 1) != hb.prob.parity) return false;
    return m2p + m2n == hb.prob.two_m;
}

// Orbits, species determinants, keys, blocks.
int make_structure(const ci_problem& p, HostBasis& hb, std::string& err)
{
    hb.prob = p;
    hb.S = std::max(top_shell(p.Z), top_shell(p.N)) + p.nmax;
    hb.orb_n.clear(); hb.orb_l.clear(); hb.orb_j2.clear(); hb.orb_m2.clear();
    for (int N = 0; N <= hb.S; N++)
        for (int l = N % 2; l <= N; l += 2)
            for (int j2 : {2 * l - 1, 2 * l + 1}) {
                if (j2 < 0) continue;
                for (int m2 = -j2; m2 <= j2; m2 += 2) {
                    hb.orb_n.push_back(N);
                    hb.orb_l.push_back(l);
                    hb.orb_j2.push_back(j2);
                    hb.orb_m2.push_back(m2);
                }
            }
    hb.nsps = (int)hb.orb_n.size();
    if (hb.nsps > 64 * kMaxWords) {
        err = "more than 256 orbits per species (shell cut " + std::to_string(hb.S) + ")";
        return CI_EUNSUPPORTED;
    }
    hb.W = (hb.nsps + 63) / 64;
    hb.N0p = lowest_quanta(p.Z);
    hb.N0n = lowest_quanta(p.N);
    hb.N0 = hb.N0p + hb.N0n;
    const int top = hb.N0 + p.nmax;

    std::vector<RawSD> raw[2];
    const int X[2] = {p.Z, p.N};
    const int other0[2] = {hb.N0n, hb.N0p};
    for (int s = 0; s < 2; s++) {
        hb.sp[s] = HostSpecies();
        hb.sp[s].X = X[s];
        hb.sp[s].budget = top - other0[s];
        enumerate_species(hb, X[s], hb.sp[s].budget, raw[s]);
    }
    // distinct keys of each species, then the keys that form a block
    std::vector<std::pair<int, int>> keys[2];
    for (int s = 0; s < 2; s++) {
        for (const RawSD& r : raw[s]) keys[s].push_back({r.nq, r.m2});
        std::sort(keys[s].begin(), keys[s].end());
        keys[s].erase(std::unique(keys[s].begin(), keys[s].end()), keys[s].end());
    }
    std::vector<char> usep(keys[0].size(), 0), usen(keys[1].size(), 0);
    for (size_t a = 0; a < keys[0].size(); a++)
        for (size_t b = 0; b < keys[1].size(); b++)
            if (block_ok(hb, keys[0][a].first, keys[0][a].second, keys[1][b].first,
                         keys[1][b].second))
                usep[a] = usen[b] = 1;
    for (int s = 0; s < 2; s++) {
        HostSpecies& sp = hb.sp[s];
        const std::vector<char>& use = s == 0 ? usep : usen;
        std::map<std::pair<int, int>, int> kid;
        for (size_t k = 0; k < keys[s].size(); k++)
            if (use[k]) {
                kid[keys[s][k]] = (int)sp.key_nq.size();
                sp.key_nq.push_back(keys[s][k].first);
                sp.key_m2.push_back(keys[s][k].second);
            }
        const int nk = sp.nk();
        std::vector<std::vector<int64_t>> members(nk);
        for (size_t r = 0; r < raw[s].size(); r++) {
            auto it = kid.find({raw[s][r].nq, raw[s][r].m2});
            if (it != kid.end()) members[it->second].push_back((int64_t)r);
        }
        sp.key_off.assign(nk + 1, 0);
        for (int k = 0; k < nk; k++) sp.key_off[k + 1] = sp.key_off[k] + (int32_t)members[k].size();
        const int W = hb.W;
        sp.sd.assign((size_t)sp.key_off[nk] * W, 0);
        sp.sd_key.assign(sp.key_off[nk], 0);
        for (int k = 0; k < nk; k++) {
            std::vector<int64_t>& m = members[k];
            std::sort(m.begin(), m.end(), [&](int64_t a, int64_t b) {
                return colex_less(raw[s][a].bits.data(), raw[s][b].bits.data(), W);
            });
            for (size_t t = 0; t < m.size(); t++) {
                int64_t g = sp.key_off[k] + (int64_t)t;
                std::memcpy(&sp.sd[g * W], raw[s][m[t]].bits.data(), W * sizeof(uint64_t));
                sp.sd_key[g] = k;
            }
        }
    }
    // blocks in (proton key, neutron key) order
    hb.blk_kp.clear(); hb.blk_kn.clear();
    hb.blk_off.assign(1, 0);
    for (int a = 0; a < hb.sp[0].nk(); a++)
        for (int b = 0; b < hb.sp[1].nk(); b++)
            if (block_ok(hb, hb.sp[0].key_nq[a], hb.sp[0].key_m2[a], hb.sp[1].key_nq[b],
                         hb.sp[1].key_m2[b])) {
                int64_t np = hb.sp[0].key_off[a + 1] - hb.sp[0].key_off[a];
                int64_t nn = hb.sp[1].key_off[b + 1] - hb.sp[1].key_off[b];
                hb.blk_kp.push_back(a);
                hb.blk_kn.push_back(b);
                hb.blk_off.push_back(hb.blk_off.back() + np * nn);
            }
    hb.dim = hb.blk_off.back();
    if (hb.dim >= (int64_t)1 << 31) {
        err = "basis dimension " + std::to_string(hb.dim) + " does not fit int32 columns";
        return CI_EUNSUPPORTED;
    }
    return CI_OK;
}

// Sectors and pair index of the two-body table.
int make_tbme_index(HostBasis& hb, std::string& err)
{
    const int n = hb.nsps;
    const ci_problem& p = hb.prob;
    int maxm = 0;
    for (int m : hb.orb_m2) maxm = std::max(maxm, m);
    hb.pair.assign((size_t)3 * n * n, kNoPair);
    hb.sec_off.clear();
    hb.sec_n.clear();
    int64_t total = 0;
    for (int cls = 0; cls < 3; cls++) {  // pp, pn, nn
        const int z = 2 - cls;            // protons in the pair
        if (p.Z - z < 0 || p.N - (2 - z) < 0) continue;
        const int n2max = hb.N0 - (lowest_quanta(p.Z - z) + lowest_quanta(p.N - (2 - z))) + p.nmax;
        for (int M = -2 * maxm; M <= 2 * maxm; M += 2)
            for (int par = 0; par < 2; par++) {
                int32_t cnt = 0;
                const int sec = (int)hb.sec_n.size();
                for (int a = 0; a < n; a++)
                    for (int b = (cls == 1 ? 0 : a + 1); b < n; b++) {
                        if (hb.orb_m2[a] + hb.orb_m2[b] != M) continue;
                        const int q = hb.orb_n[a] + hb.orb_n[b];
                        if ((q & 1) != par || q > n2max) continue;
                        if (sec >= 65536 || cnt >= 65536) {
                            err = "two-body sector too large for the pair index";
                            return CI_EUNSUPPORTED;
                        }
                        hb.pair[(size_t)cls * n * n + (size_t)a * n + b] =
                            ((uint32_t)sec << 16) | (uint32_t)cnt;
                        cnt++;
                    }
                if (cnt == 0) continue;
                hb.sec_n.push_back(cnt);
                hb.sec_off.push_back(total);
                total += (int64_t)cnt * (cnt + 1) / 2;
            }
    }
    hb.n_tbme = total;
    return CI_OK;
}

// One- and two-nucleon partner lists of every determinant of species s.
void make_partners(HostBasis& hb, int s)
{
    HostSpecies& sp = hb.sp[s];
    const int n = hb.nsps, W = hb.W, nk = sp.nk();
    const int64_t nsd = sp.nsd();
    std::unordered_map<Bits, int32_t, BitsHash> index;
    index.reserve((size_t)nsd * 2);
    for (int64_t g = 0; g < nsd; g++) {
        Bits b{};
        std::memcpy(b.data(), &sp.sd[g * W], W * sizeof(uint64_t));
        index.emplace(b, (int32_t)g);
    }
    // orbit pairs (h1 < h2) grouped by (pair 2M, parity), ascending quanta
    std::map<std::pair<int, int>, std::vector<std::pair<int16_t, int16_t>>> groups;
    for (int a = 0; a < n; a++)
        for (int b = a + 1; b < n; b++)
            groups[{hb.orb_m2[a] + hb.orb_m2[b], (hb.orb_n[a] + hb.orb_n[b]) & 1}].push_back(
                {(int16_t)a, (int16_t)b});
    for (auto& kv : groups)
        std::stable_sort(kv.second.begin(), kv.second.end(), [&](auto x, auto y) {
            return hb.orb_n[x.first] + hb.orb_n[x.second] < hb.orb_n[y.first] + hb.orb_n[y.second];
        });

    sp.seg1.assign((size_t)nsd * (nk + 1), 0);
    sp.seg12.assign((size_t)nsd * (nk + 1), 0);
    sp.self12.assign((size_t)nsd, 0);
    std::vector<int32_t> key_nq(sp.key_nq), key_m2(sp.key_m2);
    std::vector<int32_t> nq_of(nsd);
    for (int64_t g = 0; g < nsd; g++) nq_of[g] = key_nq[sp.sd_key[g]];

    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nsd < 256) nth = 1;
    std::vector<std::vector<uint64_t>> t1(nth), t12(nth);
    std::vector<std::vector<int64_t>> c1(nth), c12(nth);
    auto work = [&](unsigned t) {
        int64_t x0 = nsd * t / nth, x1 = nsd * (t + 1) / nth;
        std::vector<std::pair<int32_t, uint64_t>> L1, L12;
        std::vector<int> occ, unocc;
        for (int64_t x = x0; x < x1; x++) {
            Bits bx{};
            std::memcpy(bx.data(), &sp.sd[x * W], W * sizeof(uint64_t));
            const int kx = sp.sd_key[x];
            const int nqx = nq_of[x];
            occ.clear();
            unocc.clear();
            for (int k = 0; k < n; k++) (test_bit(bx, k) ? occ : unocc).push_back(k);
            L1.clear();
            L12.clear();
            auto same_mp = [&](int g) {
                int ky = sp.sd_key[g];
                return key_m2[ky] == key_m2[kx] && ((key_nq[ky] - key_nq[kx]) & 1) == 0;
            };
            auto local = [&](int g) { return (uint32_t)(g - sp.key_off[sp.sd_key[g]]); };
            // itself
            uint64_t self = make_rec(local((int)x), 0, 0, 0, 0, 0, false);
            L1.push_back({(int32_t)x, self});
            L12.push_back({(int32_t)x, self});
            // one nucleon: particle p (in x) -> hole h (in y)
            for (int pp : occ)
                for (int h : unocc) {
                    if (nqx - hb.orb_n[pp] + hb.orb_n[h] > sp.budget) continue;
                    Bits by = bx;
                    flip_bit(by, pp);
                    flip_bit(by, h);
                    auto it = index.find(by);
                    if (it == index.end()) continue;
                    const int g = it->second;
                    int lo = std::min(pp, h), hi = std::max(pp, h);
                    int between = count_below(bx, hi) - count_below(bx, lo + 1);
                    uint64_t r = make_rec(local(g), 1, h, pp, 0, 0, between & 1);
                    L1.push_back({g, r});
                    if (same_mp(g)) L12.push_back({g, r});
                }
            // two nucleons, same pair 2M and parity (so the key keeps its 2M
            // and the parity of its Nq)
            for (size_t u = 0; u < occ.size(); u++)
                for (size_t v = u + 1; v < occ.size(); v++) {
                    const int p1 = occ[u], p2 = occ[v];
                    auto it = groups.find({hb.orb_m2[p1] + hb.orb_m2[p2],
                                           (hb.orb_n[p1] + hb.orb_n[p2]) & 1});
                    if (it == groups.end()) continue;
                    const int room = sp.budget - nqx + hb.orb_n[p1] + hb.orb_n[p2];
                    for (auto hh : it->second) {
                        const int h1 = hh.first, h2 = hh.second;
                        if (hb.orb_n[h1] + hb.orb_n[h2] > room) break;
                        if (test_bit(bx, h1) || test_bit(bx, h2)) continue;
                        Bits by = bx;
                        flip_bit(by, p1);
                        flip_bit(by, p2);
                        flip_bit(by, h1);
                        flip_bit(by, h2);
                        auto jt = index.find(by);
                        if (jt == index.end()) continue;
                        const int g = jt->second;
                        Bits T = by;  // y without the holes = x without the particles
                        flip_bit(T, h1);
                        flip_bit(T, h2);
                        int e = count_below(by, h1) + count_below(by, h2) - 1 + count_below(T, p1) +
                                count_below(T, p2);
                        L12.push_back({g, make_rec(local(g), 2, h1, p1, h2, p2, e & 1)});
                    }
                }
            std::sort(L1.begin(), L1.end(), [](auto& a, auto& b) { return a.first < b.first; });
            std::sort(L12.begin(), L12.end(), [](auto& a, auto& b) { return a.first < b.first; });
            // segment starts per key
            int32_t* s1 = &sp.seg1[(size_t)x * (nk + 1)];
            int32_t* s12 = &sp.seg12[(size_t)x * (nk + 1)];
            size_t q1 = 0, q12 = 0;
            for (int k = 0; k <= nk; k++) {
                while (q1 < L1.size() && sp.sd_key[L1[q1].first] < k) q1++;
                while (q12 < L12.size() && sp.sd_key[L12[q12].first] < k) q12++;
                s1[k] = (int32_t)q1;
                s12[k] = (int32_t)q12;
            }
            s1[nk] = (int32_t)L1.size();
            s12[nk] = (int32_t)L12.size();
            for (size_t q = 0; q < L12.size(); q++)
                if (L12[q].first == (int32_t)x) sp.self12[x] = (int32_t)q - s12[kx];
            for (auto& e : L1) t1[t].push_back(e.second);
            for (auto& e : L12) t12[t].push_back(e.second);
            c1[t].push_back((int64_t)L1.size());
            c12[t].push_back((int64_t)L12.size());
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nth; t++) pool.emplace_back(work, t);
    work(0);
    for (auto& th : pool) th.join();

    sp.l1_ptr.assign(nsd + 1, 0);
    sp.l12_ptr.assign(nsd + 1, 0);
    int64_t x = 0;
    for (unsigned t = 0; t < nth; t++)
        for (size_t k = 0; k < c1[t].size(); k++, x++) {
            sp.l1_ptr[x + 1] = sp.l1_ptr[x] + c1[t][k];
            sp.l12_ptr[x + 1] = sp.l12_ptr[x] + c12[t][k];
        }
    sp.l1.clear();
    sp.l12.clear();
    sp.l1.reserve(sp.l1_ptr[nsd]);
    sp.l12.reserve(sp.l12_ptr[nsd]);
    for (unsigned t = 0; t < nth; t++) {
        sp.l1.insert(sp.l1.end(), t1[t].begin(), t1[t].end());
        sp.l12.insert(sp.l12.end(), t12[t].begin(), t12[t].end());
    }
}

}  // namespace

int validate_problem(const ci_problem& p, std::string& err)
{
    if (p.Z < 0 || p.N < 0 || p.Z + p.N == 0) {
        err = "need Z >= 0, N >= 0 and Z + N > 0";
        return CI_EINVAL;
    }
    if (p.Z > 40 || p.N > 40) {
        err = "Z and N above 40 are not supported";
        return CI_EUNSUPPORTED;
    }
    if (p.nmax < 0) {
        err = "nmax must be >= 0";
        return CI_EINVAL;
    }
    if (p.parity != 1 && p.parity != -1) {
        err = "parity must be +1 or -1";
        return CI_EINVAL;
    }
    if ((p.two_m + p.Z + p.N) & 1) {
        err = "two_m must have the parity of Z + N";
        return CI_EINVAL;
    }
    if (!(p.hw_mev > 0.0) || p.hw_mev > 1e6) {
        err = "hw_mev must be a positive finite energy";
        return CI_EINVAL;
    }
    return CI_OK;
}

int plan_basis(const ci_problem& p, HostBasis& hb, std::string& err)
{
    int rc = validate_problem(p, err);
    if (rc != CI_OK) return rc;
    rc = make_structure(p, hb, err);
    if (rc != CI_OK) return rc;
    rc = make_tbme_index(hb, err);
    if (rc != CI_OK) return rc;
    return CI_OK;
}

int build_basis(const ci_problem& p, HostBasis& hb, std::string& err)
{
    int rc = plan_basis(p, hb, err);
    if (rc != CI_OK) return rc;
    for (int s = 0; s < 2; s++) make_partners(hb, s);
    return CI_OK;
}

void tbme_keys(const HostBasis& hb, std::vector<int32_t>& abcd)
{
    const int n = hb.nsps;
    // pairs of each sector in table order
    std::vector<std::vector<std::pair<int, int>>> pairs(hb.sec_n.size());
    for (int cls = 0; cls < 3; cls++)
        for (int a = 0; a < n; a++)
            for (int b = 0; b < n; b++) {
                uint32_t e = hb.pair[(size_t)cls * n * n + (size_t)a * n + b];
                if (e == kNoPair) continue;
                const int ca = cls == 2 ? n + a : a;           // combined index
                const int cb = cls == 0 ? b : n + b;
                auto& v = pairs[e >> 16];
                if (v.size() <= (e & 0xffff)) v.resize((e & 0xffff) + 1);
                v[e & 0xffff] = {ca, cb};
            }
    abcd.clear();
    abcd.reserve((size_t)hb.n_tbme * 4);
    for (auto& v : pairs)
        for (size_t r = 0; r < v.size(); r++)
            for (size_t c = r; c < v.size(); c++) {
                abcd.push_back(v[r].first);
                abcd.push_back(v[r].second);
                abcd.push_back(v[c].first);
                abcd.push_back(v[c].second);
            }
}

}  // namespace ci
