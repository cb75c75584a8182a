// Host construction of the basis indexing of one problem (paper Sec. 2: the
// indexing systems of the many-body basis are set up before the matrix is
// built; Sec. 5.2: index structures are built contiguously on the host and
// moved to the device with one allocation and one copy).
//
// Builds: the oscillator orbits; the proton and neutron determinants grouped
// by (Nq, 2M) key; the compatible key blocks and row offsets; the sector /
// pair index of the two-body table; all flat, for a single upload.  The
// partner lists of the determinants are built on the device.
#include <algorithm>
#include <array>
#include <cstring>
#include <map>

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

inline void flip_bit(Bits& b, int k) { b[k >> 6] ^= 1ull << (k & 63); }

// Visits every X-orbit determinant with Nq <= budget in colex order (as
// unsigned W-word integers, word W-1 most significant): the highest orbit is
// chosen first, in ascending order, and the rest recursively below it.  low[j]
// is the fewest quanta j nucleons can have.  visit(bits, nq, 2M).
template <class F>
void colex_visit(const HostBasis& hb, int left, int limit, int nq, int m2, int budget, const int* low, Bits& cur,
                 F& visit)
{
    if (left == 0) {
        visit(cur, nq, m2);
        return;
    }
    for (int k = left - 1; k < limit; k++) {
        // orbits ascend in N: a larger top orbit never costs less
        if (nq + hb.orb_n[k] + low[left - 1] > budget) break;
        flip_bit(cur, k);
        colex_visit(hb, left - 1, k, nq + hb.orb_n[k], m2 + hb.orb_m2[k], budget, low, cur, visit);
        flip_bit(cur, k);
    }
}

template <class F>
void visit_species(const HostBasis& hb, int X, int budget, F& visit)
{
    std::vector<int> low(X + 1);
    for (int j = 0; j <= X; j++) low[j] = lowest_quanta(j);
    Bits cur{};
    colex_visit(hb, X, hb.nsps, 0, 0, budget, low.data(), cur, visit);
}

bool block_ok(const HostBasis& hb, int nqp, int m2p, int nqn, int m2n)
{
    int nq = nqp + nqn;
    if (nq > hb.N0 + hb.prob.nmax) return false;
    if (((nq & 1) ? -1 : 1) != hb.prob.parity) return false;
    return m2p + m2n == hb.prob.two_m;
}

// Oscillator orbits and the lowest filling.
int make_orbits(const ci_problem& p, HostBasis& hb, std::string& err)
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
    return CI_OK;
}

// Species determinants, keys, blocks (the orbits are set).
int make_determinants(HostBasis& hb, std::string& err)
{
    const ci_problem& p = hb.prob;
    const int top = hb.N0 + p.nmax;

    // keys (Nq, 2M) of each species on a dense grid
    int maxm = 0;
    for (int m : hb.orb_m2) maxm = std::max(maxm, m);
    const int mtot = std::max(1, std::max(p.Z, p.N)) * maxm;  // |2M| bound of one species
    const int nqs = top + 1, nms = 2 * mtot + 1;
    auto cell = [&](int nq, int m2) { return nq * nms + (m2 + mtot); };
    const int X[2] = {p.Z, p.N};
    const int other0[2] = {hb.N0n, hb.N0p};
    // protons and neutrons of an N = Z problem have the same determinants
    const bool twin = p.Z == p.N;
    std::vector<int32_t> present[2];
    for (int s = 0; s < 2; s++) {
        hb.sp[s] = HostSpecies();
        hb.sp[s].X = X[s];
        hb.sp[s].budget = top - other0[s];
        if (s == 1 && twin) {
            present[1] = present[0];
            continue;
        }
        present[s].assign((size_t)nqs * nms, 0);
        std::vector<int32_t>& pr = present[s];
        auto count = [&](const Bits&, int nq, int m2) { pr[cell(nq, m2)]++; };
        visit_species(hb, X[s], hb.sp[s].budget, count);
    }
    // keep the keys that take part in a block
    std::vector<char> use[2];
    use[0].assign((size_t)nqs * nms, 0);
    use[1].assign((size_t)nqs * nms, 0);
    for (int qa = 0; qa < nqs; qa++)
        for (int ma = -mtot; ma <= mtot; ma++) {
            if (!present[0][cell(qa, ma)]) continue;
            const int mb = p.two_m - ma;
            if (mb < -mtot || mb > mtot) continue;
            for (int qb = 0; qb < nqs; qb++)
                if (present[1][cell(qb, mb)] && block_ok(hb, qa, ma, qb, mb))
                    use[0][cell(qa, ma)] = use[1][cell(qb, mb)] = 1;
        }
    for (int s = 0; s < 2; s++) {
        HostSpecies& sp = hb.sp[s];
        if (s == 1 && twin) {
            const int budget = sp.budget;
            sp = hb.sp[0];
            sp.X = X[1];
            sp.budget = budget;
            continue;
        }
        // key ids in (Nq, 2M) order
        std::vector<int32_t> kid((size_t)nqs * nms, -1);
        for (int q = 0; q < nqs; q++)
            for (int m = -mtot; m <= mtot; m++)
                if (use[s][cell(q, m)]) {
                    kid[cell(q, m)] = (int32_t)sp.key_nq.size();
                    sp.key_nq.push_back(q);
                    sp.key_m2.push_back(m);
                }
        const int nk = sp.nk();
        sp.key_off.assign(nk + 1, 0);
        int64_t tot = 0;
        for (int k = 0; k < nk; k++) {
            const int64_t n = present[s][cell(sp.key_nq[k], sp.key_m2[k])];
            // partner records hold a determinant's position in its key in 24 bits
            if (n > (int64_t)kRecLocalMask + 1) {
                err = "a species key holds more than 2^24 determinants";
                return CI_EUNSUPPORTED;
            }
            tot += n;
            if (tot >= ((int64_t)1 << 31)) {
                err = "more than 2^31 determinants of one species";
                return CI_EUNSUPPORTED;
            }
            sp.key_off[k + 1] = (int32_t)tot;
        }
        const int W = hb.W;
        sp.sd.resize((size_t)sp.key_off[nk] * W);
        sp.sd_key.resize(sp.key_off[nk]);
        // second visit: each determinant goes to the next slot of its key, so
        // every key's run is in colex order
        std::vector<int32_t> fillp(sp.key_off.begin(), sp.key_off.end() - 1);
        uint64_t* sdp = sp.sd.data();
        int32_t* skp = sp.sd_key.data();
        auto place = [&](const Bits& bits, int nq, int m2) {
            const int k = kid[cell(nq, m2)];
            if (k < 0) return;
            const int32_t g = fillp[k]++;
            for (int w = 0; w < W; w++) sdp[(size_t)g * W + w] = bits[w];
            skp[g] = k;
        };
        visit_species(hb, X[s], sp.budget, place);
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

// Sectors and pair index of the two-body table: sectors ordered by class
// (pp, pn, nn), pair 2M, pair parity; pairs lexicographic inside a sector.
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
        // sectors of this class on a dense (2M, parity) grid: count, number in
        // (2M, parity) order, then give each pair its lexicographic position
        const int nm = 4 * maxm + 1;
        std::vector<int32_t> cnt(2 * nm, 0), sid(2 * nm, -1);
        auto valid = [&](int a, int b) { return hb.orb_n[a] + hb.orb_n[b] <= n2max; };
        auto slot = [&](int a, int b) {
            return (hb.orb_m2[a] + hb.orb_m2[b] + 2 * maxm) * 2 + ((hb.orb_n[a] + hb.orb_n[b]) & 1);
        };
        // orbits ascend in N, so the valid partners b of a are a prefix of the
        // loop and the search stops at the first invalid one
        for (int a = 0; a < n; a++)
            for (int b = (cls == 1 ? 0 : a + 1); b < n && valid(a, b); b++) cnt[slot(a, b)]++;
        for (int t = 0; t < 2 * nm; t++) {
            if (!cnt[t]) continue;
            const int sec = (int)hb.sec_n.size();
            if (sec >= 65536 || cnt[t] > 65536) {
                err = "two-body sector too large for the pair index";
                return CI_EUNSUPPORTED;
            }
            sid[t] = sec;
            hb.sec_n.push_back(cnt[t]);
            hb.sec_off.push_back(total);
            total += (int64_t)cnt[t] * (cnt[t] + 1) / 2;
            cnt[t] = 0;  // reused as the running position
        }
        for (int a = 0; a < n; a++)
            for (int b = (cls == 1 ? 0 : a + 1); b < n && valid(a, b); b++) {
                const int t = slot(a, b);
                hb.pair[(size_t)cls * n * n + (size_t)a * n + b] = ((uint32_t)sid[t] << 16) | (uint32_t)cnt[t]++;
            }
    }
    hb.n_tbme = total;
    if (total >= ((int64_t)1 << 31)) {
        err = "two-body table of " + std::to_string(total) + " entries does not fit int32 indices";
        return CI_EUNSUPPORTED;
    }
    return CI_OK;
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
    if (p.kinetic != 0 && p.kinetic != 1) {
        err = "kinetic must be 0 or 1";
        return CI_EINVAL;
    }
    if (!(p.hw_mev > 0.0) || p.hw_mev > 1e6) {
        err = "hw_mev must be a positive finite energy";
        return CI_EINVAL;
    }
    return CI_OK;
}

int plan_orbits(const ci_problem& p, HostBasis& hb, std::string& err)
{
    int rc = validate_problem(p, err);
    if (rc != CI_OK) return rc;
    return make_orbits(p, hb, err);
}

int plan_determinants(HostBasis& hb, std::string& err) { return make_determinants(hb, err); }

int plan_tbme_index(HostBasis& hb, std::string& err) { return make_tbme_index(hb, err); }

int plan_basis(const ci_problem& p, HostBasis& hb, std::string& err)
{
    int rc = plan_orbits(p, hb, err);
    if (rc == CI_OK) rc = make_determinants(hb, err);
    if (rc != CI_OK) return rc;
    return plan_tbme_index(hb, err);
}

void write_pair64(const HostBasis& hb, uint64_t* out)
{
    // device form: the entry also carries the row base of the pair
    const size_t n = hb.pair.size();
    for (size_t t = 0; t < n; t++) {
        const uint32_t e = hb.pair[t];
        if (e == kNoPair) {
            out[t] = kNoPair64;
            continue;
        }
        const int64_t sec = e >> 16, r = e & 0xffff, ns = hb.sec_n[sec];
        const int64_t base = hb.sec_off[sec] + r * (2 * ns - r + 1) / 2 - r;
        out[t] = ((uint64_t)(uint32_t)base << 32) | e;
    }
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
