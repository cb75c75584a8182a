// C ABI of libci (declared in include/ci.h): validation, the basis handle,
// the device index tables, and the launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "ci_internal.h"
#include "threebody.h"

namespace ci {
hipError_t launch_count(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                        int64_t* row_ptr, int64_t nrp, const int64_t* seg_first, int64_t* scan_tmp,
                        const ci_tuning& t, unsigned long long* queue, int full, hipStream_t s);
hipError_t launch_nnz(const int64_t* row_ptr, const int64_t* first, const int64_t* last, int64_t* nnz,
                      int n, hipStream_t s);
hipError_t launch_fill(const BasisDev* bases, int nb, const int64_t* basis_row0, int64_t nrows,
                       const float* tbme, const int64_t* row_ptr, int64_t nrp, int32_t* col, float* val,
                       uint32_t* keys, const ci_tuning& t, unsigned long long* queue, int full, hipStream_t s);
hipError_t launch_vjp(const BasisDev* bases, int nbases, const int32_t* blk_basis, const int32_t* blk_local,
                      int nblocks, int64_t ntiles, int64_t* tile_off, AdjBasis* adjb, int64_t nbuckets, int chunks,
                      unsigned long long* part,
                      int64_t nrows, const int64_t* row_ptr, int64_t nrp, const float* gval, const uint32_t* keys,
                      float* gtbme, unsigned long long* gacc, uint64_t* recs, int64_t rec_cap,
                      unsigned long long* rec_count, int32_t* hist, int64_t ntbme, const ci_tuning& t,
                      unsigned long long* queue, unsigned long long* gscale, int64_t nnz_total, hipStream_t s);
int adjoint_slots(bool wide);
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch(void** p);
hipError_t launch_inclusive_scan(int64_t* x, int64_t n, int64_t* tmp, hipStream_t s);
hipError_t launch_copy_i64(const int64_t* src, int64_t* dst, hipStream_t s);
hipError_t launch_partner_count(const PartnerArgs& a, hipStream_t s);
hipError_t launch_partner_fill(const PartnerArgs& a, int64_t n1, int64_t n12, hipStream_t s);
hipError_t run_probes(void* buf, size_t bytes, hipStream_t s, double* store_bps, double* steps_per_s);
hipError_t launch_spmv(const int64_t* row_ptr, const int32_t* col, const float* val, const double* x, double* y,
                       int64_t nrows, hipStream_t s);
hipError_t launch_spmv_upper(const int64_t* row_ptr, const int32_t* col, const float* val, const double* x,
                             double* y, int64_t nrows, hipStream_t s);
size_t lanczos_work_bytes(int64_t dim, int max_iter);
hipError_t launch_h3_rows(const BasisDev* bases, const int64_t* dims, const int* words, const void* const* index,
                          int nb, const float* tbme, int v3_kind, uint64_t v3_seed, double v3_scale, int64_t* row_ptr,
                          int32_t* col, float* val, bool fill, int full, hipStream_t s);
hipError_t launch_h3_index(bool fill, const BasisDev* B, int species, int64_t nsd, int W, int32_t* seg, int64_t* ptr,
                           uint64_t* rec, hipStream_t s);
hipError_t run_lanczos(const int64_t* row_ptr, const int32_t* col, const float* val, int64_t D, const double* x0,
                       int max_iter, double tol, double* eval, int* iters, double* evec, void* work, hipStream_t s,
                       bool upper);
}  // namespace ci

using namespace ci;

static thread_local std::string g_err;

static int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

static int hip_fail(hipError_t e, const char* where)
{
    return fail(CI_EHIP, std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

// ---------------------------------------------------------------------------
// Per-thread pinned staging buffer of the host-written tables and the
// descriptors (host memory, grown as needed and kept): copies out of pinned
// memory are asynchronous, so the host goes on while they run.  A build
// returns before its last copy out of the buffer has run; an event recorded
// after that copy is waited on before the buffer is written again.
struct StagingFence {
    hipEvent_t ev = nullptr;
    int device = -1;
    bool pending = false;
};
static thread_local StagingFence t_fence;

static hipError_t staging_wait()
{
    if (!t_fence.pending) return hipSuccess;
    t_fence.pending = false;
    return hipEventSynchronize(t_fence.ev);
}

static hipError_t staging_fence(hipStream_t s, int device)
{
    if (!t_fence.ev || t_fence.device != device) {
        if (t_fence.ev) (void)hipEventDestroy(t_fence.ev);
        t_fence.ev = nullptr;
        hipError_t e = hipEventCreateWithFlags(&t_fence.ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        t_fence.device = device;
    }
    hipError_t e = hipEventRecord(t_fence.ev, s);
    if (e != hipSuccess) return e;
    t_fence.pending = true;
    return hipSuccess;
}

// A second stream per device (default priority) for host-to-device copies
// that overlap the kernels of the caller's stream, created on first use and
// kept until the process ends; the caller's stream waits for such a copy
// through a per-thread event before it uses the data.
static hipError_t copy_stream(int device, hipStream_t* out)
{
    static std::mutex mu;
    static std::map<int, hipStream_t> streams;
    std::lock_guard<std::mutex> g(mu);
    auto it = streams.find(device);
    if (it != streams.end()) {
        *out = it->second;
        return hipSuccess;
    }
    hipStream_t st = nullptr;
    const hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    streams[device] = st;
    *out = st;
    return hipSuccess;
}

static thread_local StagingFence t_copy_done;

// Copies bytes host -> device on the device's copy stream and makes stream s
// wait for the copy.
static hipError_t copy_beside(void* dst, const void* src, size_t bytes, hipStream_t s, int device)
{
    hipStream_t cs = nullptr;
    hipError_t e = copy_stream(device, &cs);
    if (e != hipSuccess) return e;
    if (!t_copy_done.ev || t_copy_done.device != device) {
        if (t_copy_done.ev) (void)hipEventDestroy(t_copy_done.ev);
        t_copy_done.ev = nullptr;
        e = hipEventCreateWithFlags(&t_copy_done.ev, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        t_copy_done.device = device;
    }
    e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipEventRecord(t_copy_done.ev, cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, t_copy_done.ev, 0);
    return e;
}

static char* pinned_staging(size_t bytes)
{
    struct Buf {
        char* p = nullptr;
        size_t n = 0;
    };
    static thread_local Buf b;
    if (staging_wait() != hipSuccess) return nullptr;
    if (b.n < bytes) {
        if (b.p) (void)hipHostFree(b.p);
        b.p = nullptr;
        b.n = 0;
        const size_t cap = std::max(bytes, (size_t)1 << 20);
        if (hipHostMalloc((void**)&b.p, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
        b.n = cap;
    }
    return b.p;
}

// Per-thread pinned buffer for the nnz counts the count passes read back
// (they synchronize before returning, so the buffer is free again).
static int64_t* pinned_counts(size_t n)
{
    struct Buf {
        int64_t* p = nullptr;
        size_t n = 0;
    };
    static thread_local Buf b;
    if (b.n < n) {
        if (b.p) (void)hipHostFree(b.p);
        b.p = nullptr;
        b.n = 0;
        const size_t cap = std::max<size_t>(n, 4096);
        if (hipHostMalloc((void**)&b.p, cap * sizeof(int64_t), hipHostMallocDefault) != hipSuccess) return nullptr;
        b.n = cap;
    }
    return b.p;
}
namespace {

// Bump layout (256-byte aligned pieces) of one device allocation.
struct Layout {
    size_t off = 0;
    template <typename T>
    size_t take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        size_t o = off;
        off += count * sizeof(T);
        return o;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

using Key = std::tuple<int, int, int, int, int, double, int>;

Key key_of(const ci_problem& p) { return Key(p.Z, p.N, p.nmax, p.two_m, p.parity, p.hw_mev, p.kinetic); }

void fill_info(const HostBasis& hb, ci_basis_info& in)
{
    std::memset(&in, 0, sizeof in);
    in.shell_max = hb.S;
    in.n_sps = hb.nsps;
    in.n_words = hb.W;
    in.n0 = hb.N0;
    in.n_pkeys = hb.sp[0].nk();
    in.n_nkeys = hb.sp[1].nk();
    in.n_blocks = hb.nblk();
    in.n_sectors = (int32_t)hb.sec_n.size();
    in.n_psd = hb.sp[0].nsd();
    in.n_nsd = hb.sp[1].nsd();
    in.dim = hb.dim;
    in.n_tbme = hb.n_tbme;
}

// offsets of one species' tables in the arena
struct SpOff {
    size_t sd, sdT, sd_key, key_off, key_nq, key_m2, l1_ptr, l12_ptr, seg1, seg12, self12;
};
struct UOff {
    SpOff sp[2];
    size_t blk_kp, blk_kn, blk_off, blk, pair, orb_n, orb_qn, totals;
    size_t bytes;
};

// Equal determinant tables (same orbits, words, keys and determinants) have
// equal partner lists.
bool same_species(const HostBasis& A, int sa, const HostBasis& B, int sb)
{
    const HostSpecies& a = A.sp[sa];
    const HostSpecies& b = B.sp[sb];
    return A.nsps == B.nsps && A.W == B.W && a.X == b.X && a.key_off == b.key_off && a.key_nq == b.key_nq &&
           a.key_m2 == b.key_m2 && a.sd == b.sd;
}

// The two-body pair indexes of the unique problems of a build, on a helper
// thread (they need only the orbits, and the calling thread meanwhile
// enumerates the determinants and starts the device); once the calling
// thread names where the device form goes (set_targets), the helper writes it
// there too.  The destructor joins, so every return path of the build waits
// for the thread.
class PairIndexer {
public:
    explicit PairIndexer(const std::vector<std::shared_ptr<HostBasis>>& ub)
        : ub_(ub), rc_(ub.size(), CI_OK), err_(ub.size())
    {
        std::future<std::vector<uint64_t*>> dst = dst_.get_future();
        try {
            th_ = std::thread([this](std::future<std::vector<uint64_t*>> d) {
                index_all();
                write_all(d.get());  // empty: the build gave up
            }, std::move(dst));
        } catch (...) {
            inline_ = true;  // no thread to be had: the same work on the calling thread
            index_all();
        }
    }
    ~PairIndexer()
    {
        release({});
        if (th_.joinable()) th_.join();
    }
    // Where the device form of each problem's index goes (host memory that
    // stays valid until wait() returns).
    void set_targets(const std::vector<uint64_t*>& out) { release(out); }
    // Joins; CI_OK, or the first failure with its problem's position and message.
    int wait(size_t* bad, std::string& err)
    {
        release({});
        if (th_.joinable()) th_.join();
        for (size_t u = 0; u < ub_.size(); u++)
            if (rc_[u] != CI_OK) {
                *bad = u;
                err = err_[u];
                return rc_[u];
            }
        return CI_OK;
    }

private:
    void index_all()
    {
        for (size_t u = 0; u < ub_.size(); u++) rc_[u] = plan_tbme_index(*ub_[u], err_[u]);
    }
    void write_all(const std::vector<uint64_t*>& out)
    {
        for (size_t u = 0; u < out.size() && u < ub_.size(); u++)
            if (rc_[u] == CI_OK) write_pair64(*ub_[u], out[u]);
    }
    void release(const std::vector<uint64_t*>& out)
    {
        if (sent_) return;
        sent_ = true;
        if (inline_)
            write_all(out);
        else
            dst_.set_value(out);
    }
    std::vector<std::shared_ptr<HostBasis>> ub_;
    std::vector<int> rc_;
    std::vector<std::string> err_;
    std::promise<std::vector<uint64_t*>> dst_;
    bool sent_ = false;
    bool inline_ = false;
    std::thread th_;
};

}  // namespace

namespace {

// Mean time (ms) of reps runs of f on stream s after one warm-up run.
template <typename F>
int time_ms(F f, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms)
{
    hipError_t e = f();
    for (int r = 0; r <= reps && e == hipSuccess; r++) {
        if (r == 1) e = hipEventRecord(e0, s);
        if (e == hipSuccess && r > 0) e = f();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    *ms /= (float)reps;
    return CI_OK;
}

}  // namespace

// Process-wide cache of tuned launch shapes, keyed by the problem list.
namespace {
std::mutex g_tune_mu;
std::map<std::vector<std::tuple<int, int, int, int, int, double, int>>, ci_tuning> g_tune;

std::vector<std::tuple<int, int, int, int, int, double, int>> tune_key(const std::vector<ci_problem>& p)
{
    std::vector<std::tuple<int, int, int, int, int, double, int>> k;
    for (const ci_problem& q : p) k.emplace_back(q.Z, q.N, q.nmax, q.two_m, q.parity, q.hw_mev, q.kinetic);
    return k;
}

ci_tuning default_tuning() { return ci_tuning{4, 0, 64, 8, 1, 96, 8, 1, 0, 0, 0}; }

ci_tuning cached_tuning(const std::vector<ci_problem>& p)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(tune_key(p));
    return it == g_tune.end() ? default_tuning() : it->second;
}

void remember_tuning(const std::vector<ci_problem>& p, const ci_tuning& t)
{
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[tune_key(p)] = t;
}
}  // namespace
// The handle.  Its device memory is the caller's: the index tables live in
// the arena given to ci_basis_build, the partner lists in the memory given to
// ci_basis_build_lists; the library neither allocates nor frees device memory
// for the two-body path.  Host memory: the planned tables of each problem.
struct ci_basis {
    int device = 0;
    std::vector<ci_basis_info> info;
    std::vector<std::shared_ptr<HostBasis>> host;  // per problem (shared for equal problems)
    char* arena = nullptr;                         // caller's: index tables
    char* lists = nullptr;                         // caller's: partner lists
    size_t arena_bytes = 0, list_bytes = 0;
    bool lists_counted = false;  // ci_basis_list_bytes has read the list lengths
    bool ready = false;          // ci_basis_build_lists has placed the lists
    // what the partner lists need after the build
    std::vector<std::shared_ptr<HostBasis>> uniq;  // unique problems
    std::vector<int> which;                        // problem -> unique problem
    std::vector<int> canon;                        // species table 2u + s -> first equal table
    std::vector<UOff> uo;                          // offsets of the unique problems' tables in the arena
    std::vector<int64_t> totals;                   // list lengths (l1, l12) per species table
    std::vector<size_t> lo1, lo12;                 // list offsets in the list memory
    std::vector<BasisDev> bd;                      // descriptors (list pointers set when placed)
    BasisDev* d_bases = nullptr;
    int64_t* d_basis_row0 = nullptr;  // first global row of each basis, [n + 1]
    int64_t nrows = 0;                // sum of the dimensions
    int64_t* d_seg_first = nullptr;   // R_b
    int64_t* d_seg_last = nullptr;    // R_b + D_b
    int64_t* d_scan_tmp = nullptr;
    int64_t* d_nnz = nullptr;
    unsigned long long* d_queue = nullptr;  // work counter of the persistent launches
    int32_t* d_blk_basis = nullptr;         // global block list of the batch: problem, local block
    int32_t* d_blk_local = nullptr;
    int64_t* d_tile_off = nullptr;          // adjoint tiles per block (inclusive scan), [nblocks + 1]
    AdjBasis* d_adjb = nullptr;             // per-basis layout of the adjoint's tile records
    unsigned long long* d_rec_count = nullptr;  // records written by the adjoint's tiles
    unsigned long long* d_gscale = nullptr;     // per basis: the adjoint's fixed-point scale (max |G|, then the shift)
    mutable int64_t nnz_total = -1;         // stored entries of all bases (after the upper-triangle count)
    int nblocks = 0;
    ci_tuning tune{};
    std::vector<ci_problem> probs;          // key of the process-wide tuning cache
    int64_t n_rowptr = 0;
    int64_t n_tbme = 0;
    // three-body partner indexes (built on first use; library allocations):
    // per basis (seg, ptr, rec) device pointers, and the allocations
    std::vector<const void*> h3_index;
    std::vector<void*> h3_mem;
    ~ci_basis()
    {
        for (void* m : h3_mem) (void)hipFree(m);
    }
};

namespace {

// Host plan of one build and the layout of its arena.  The size query of
// ci_basis_build makes it and keeps it for the calling thread, so that the
// build that follows with the same problems does not plan again.
struct BuildPlan {
    std::vector<Key> keys;  // the problem list
    std::vector<ci_problem> probs;
    std::vector<int> which;
    std::vector<std::shared_ptr<HostBasis>> ub;
    std::unique_ptr<PairIndexer> pairs;  // two-body pair indexes, on a helper thread
    std::vector<int> canon;
    std::vector<UOff> uo;
    size_t pair_start = 0, host_bytes = 0;
    size_t o_row0 = 0, o_first = 0, o_last = 0, o_blk_basis = 0, o_blk_local = 0;
    size_t o_bases = 0, o_scan = 0, o_nnz = 0, o_queue = 0, o_rec_count = 0, o_gscale = 0, o_tile_off = 0, o_adjb = 0;
    size_t bytes = 0;
    int nblocks = 0;
};

thread_local std::unique_ptr<BuildPlan> t_pending;

std::vector<Key> keys_of(const ci_problem* probs, int32_t n)
{
    std::vector<Key> k;
    for (int32_t b = 0; b < n; b++) k.push_back(key_of(probs[b]));
    return k;
}

// Validates and plans the problems (orbits, then the pair indexes on a helper
// thread while the determinants are enumerated here) and lays out the arena.
int plan_build(const ci_problem* probs, int32_t n_probs, BuildPlan& P, std::string& err)
{
    P.keys = keys_of(probs, n_probs);
    P.probs.assign(probs, probs + n_probs);
    std::map<Key, int> uniq;
    P.which.assign(n_probs, 0);
    for (int32_t b = 0; b < n_probs; b++) {
        int rc = validate_problem(probs[b], err);
        if (rc != CI_OK) return err = "problem " + std::to_string(b) + ": " + err, rc;
        auto it = uniq.find(P.keys[b]);
        if (it != uniq.end()) {
            P.which[b] = it->second;
            continue;
        }
        auto hb = std::make_shared<HostBasis>();
        rc = plan_orbits(probs[b], *hb, err);
        if (rc != CI_OK) return err = "problem " + std::to_string(b) + ": " + err, rc;
        P.which[b] = (int)P.ub.size();
        uniq[P.keys[b]] = P.which[b];
        P.ub.push_back(hb);
    }
    P.pairs.reset(new PairIndexer(P.ub));
    for (size_t u = 0; u < P.ub.size(); u++) {
        const int rc = plan_determinants(*P.ub[u], err);
        if (rc != CI_OK) return err = "problem " + std::to_string(u) + ": " + err, rc;
    }
    // Species tables with equal content (protons and neutrons of an N = Z
    // nucleus, or one species shared by several problems of a batch) are
    // stored once and get their partner lists once: canon[2u + s] is the
    // first equal species table.
    const std::vector<std::shared_ptr<HostBasis>>& ub = P.ub;
    const int nsp = 2 * (int)ub.size();
    P.canon.assign(nsp, 0);
    for (int i = 0; i < nsp; i++) {
        P.canon[i] = i;
        for (int j = 0; j < i; j++)
            if (P.canon[j] == j && same_species(*ub[i / 2], i % 2, *ub[j / 2], j % 2)) {
                P.canon[i] = j;
                break;
            }
    }
    // Arena: tables the host writes first (mirrored and copied up), then the
    // tables the device computes (never copied).
    Layout L;
    P.uo.assign(ub.size(), UOff{});
    std::vector<size_t> ubytes(ub.size(), 0);
    int64_t max_scan = 1;
    for (size_t u = 0; u < ub.size(); u++) {
        const HostBasis& hb = *ub[u];
        for (int sidx = 0; sidx < 2; sidx++) {
            if (P.canon[2 * u + sidx] != (int)(2 * u + sidx)) continue;
            const HostSpecies& sp = hb.sp[sidx];
            SpOff& o = P.uo[u].sp[sidx];
            const size_t nsd = (size_t)sp.nsd(), nk = (size_t)sp.nk();
            const size_t s0 = L.off;
            o.sd = L.take<uint64_t>(sp.sd.size());
            o.sdT = L.take<uint64_t>(sp.sd.size());
            o.sd_key = L.take<int32_t>(nsd);
            o.key_off = L.take<int32_t>(nk + 1);
            o.key_nq = L.take<int32_t>(nk);
            o.key_m2 = L.take<int32_t>(nk);
            ubytes[u] += L.off - s0;
        }
        const size_t s0 = L.off;
        P.uo[u].blk_kp = L.take<int32_t>(hb.blk_kp.size());
        P.uo[u].blk_kn = L.take<int32_t>(hb.blk_kn.size());
        P.uo[u].blk_off = L.take<int64_t>(hb.blk_off.size());
        P.uo[u].blk = L.take<BlockInfo>(hb.blk_kp.size());
        P.uo[u].orb_n = L.take<int32_t>(hb.orb_n.size());
        P.uo[u].orb_qn = L.take<int32_t>(hb.orb_n.size());
        ubytes[u] += L.off - s0;
    }
    P.o_row0 = L.take<int64_t>(n_probs + 1);
    P.o_first = L.take<int64_t>(n_probs);
    P.o_last = L.take<int64_t>(n_probs);
    P.nblocks = 0;
    for (int32_t b = 0; b < n_probs; b++) P.nblocks += ub[P.which[b]]->nblk();
    P.o_blk_basis = L.take<int32_t>(std::max(P.nblocks, 1));
    P.o_blk_local = L.take<int32_t>(std::max(P.nblocks, 1));
    // the pair indices last: they are written after the partner kernels start
    P.pair_start = L.off;
    for (size_t u = 0; u < ub.size(); u++) {
        const size_t n = (size_t)ub[u]->nsps;
        P.uo[u].pair = L.take<uint64_t>(3 * n * n);
        ubytes[u] += 3 * n * n * sizeof(uint64_t);
    }
    P.host_bytes = L.off;
    for (size_t u = 0; u < ub.size(); u++) {
        const HostBasis& hb = *ub[u];
        for (int sidx = 0; sidx < 2; sidx++) {
            const int c = P.canon[2 * u + sidx];
            SpOff& o = P.uo[u].sp[sidx];
            if (c != (int)(2 * u + sidx)) {
                o = P.uo[c / 2].sp[c % 2];
                continue;
            }
            const HostSpecies& sp = hb.sp[sidx];
            const size_t nsd = (size_t)sp.nsd(), nk = (size_t)sp.nk();
            const size_t s0 = L.off;
            o.l1_ptr = L.take<int64_t>(nsd + 1);
            o.l12_ptr = L.take<int64_t>(nsd + 1);
            o.seg1 = L.take<int32_t>(nsd * (nk + 1));
            o.seg12 = L.take<int32_t>(nsd * (nk + 1));
            o.self12 = L.take<int32_t>(nsd);
            ubytes[u] += L.off - s0;
            max_scan = std::max<int64_t>(max_scan, (int64_t)nsd + 1);
        }
        P.uo[u].totals = L.take<int64_t>(4);  // list lengths: l1, l12 of each species
        P.uo[u].bytes = ubytes[u];
    }
    int64_t R = 0;
    for (int32_t b = 0; b < n_probs; b++) R += ub[P.which[b]]->dim + 1;
    max_scan = std::max(max_scan, R);
    P.o_bases = L.take<BasisDev>(n_probs);
    P.o_scan = L.take<int64_t>((max_scan + 4095) / 4096 + 1);
    P.o_nnz = L.take<int64_t>(n_probs);
    P.o_queue = L.take<unsigned long long>(1);
    P.o_rec_count = L.take<unsigned long long>(1);
    P.o_gscale = L.take<unsigned long long>(n_probs);
    P.o_tile_off = L.take<int64_t>(P.nblocks + 1);
    P.o_adjb = L.take<AdjBasis>(n_probs);
    P.bytes = L.bytes();
    return CI_OK;
}

// Arguments of the partner-list kernels of unique problem u, species sidx.
PartnerArgs partner_args(const ci_basis& h, size_t u, int sidx)
{
    const HostSpecies& sp = h.uniq[u]->sp[sidx];
    const SpOff& o = h.uo[u].sp[sidx];
    char* dev = h.arena;
    PartnerArgs a{};
    a.sd = (const uint64_t*)(dev + o.sd);
    a.sdT = (const uint64_t*)(dev + o.sdT);
    a.sd_key = (const int32_t*)(dev + o.sd_key);
    a.key_off = (const int32_t*)(dev + o.key_off);
    a.key_nq = (const int32_t*)(dev + o.key_nq);
    a.key_m2 = (const int32_t*)(dev + o.key_m2);
    a.l1_ptr = (int64_t*)(dev + o.l1_ptr);
    a.l12_ptr = (int64_t*)(dev + o.l12_ptr);
    a.seg1 = (int32_t*)(dev + o.seg1);
    a.seg12 = (int32_t*)(dev + o.seg12);
    a.self12 = (int32_t*)(dev + o.self12);
    a.nsd = (int32_t)sp.nsd();
    a.nk = sp.nk();
    a.W = h.uniq[u]->W;
    return a;
}

int need_ready(const ci_basis* b)
{
    if (!b) return fail(CI_EINVAL, "null pointer");
    if (!b->ready) return fail(CI_EINVAL, "the basis has no partner lists yet (ci_basis_list_bytes, ci_basis_build_lists)");
    return CI_OK;
}

}  // namespace

extern "C" {

const char* ci_last_error(void) { return g_err.c_str(); }

int ci_basis_plan(const ci_problem* probs, int32_t n_probs, ci_basis_info* info)
{
    if (!probs || !info || n_probs <= 0) return fail(CI_EINVAL, "null pointer or n_probs <= 0");
    std::string err;
    BuildPlan P;
    int rc = plan_build(probs, n_probs, P, err);
    if (rc != CI_OK) return fail(rc, err);
    size_t bad = 0;
    rc = P.pairs->wait(&bad, err);
    if (rc != CI_OK) return fail(rc, "problem " + std::to_string(bad) + ": " + err);
    int64_t R = 0, T = 0;
    for (int32_t b = 0; b < n_probs; b++) {
        const HostBasis& hb = *P.ub[P.which[b]];
        fill_info(hb, info[b]);
        info[b].row_ptr_offset = R;
        info[b].tbme_offset = T;
        info[b].index_bytes = -1;  // known after the partner lists are counted
        info[b].arena_bytes = (int64_t)P.bytes;
        info[b].list_bytes = -1;
        R += hb.dim + 1;
        T += hb.n_tbme;
    }
    return CI_OK;
}

int ci_tbme_keys(const ci_problem* prob, int32_t* abcd, int64_t cap)
{
    if (!prob || (!abcd && cap > 0)) return fail(CI_EINVAL, "null pointer");
    std::string err;
    HostBasis hb;
    int rc = plan_basis(*prob, hb, err);
    if (rc != CI_OK) return fail(rc, err);
    if (cap < hb.n_tbme) return fail(CI_ESPACE, "need room for " + std::to_string(hb.n_tbme) + " keys");
    std::vector<int32_t> k;
    tbme_keys(hb, k);
    std::memcpy(abcd, k.data(), k.size() * sizeof(int32_t));
    return CI_OK;
}

int ci_basis_build(const ci_problem* probs, int32_t n_probs, ci_basis_info* info, void* arena,
                   size_t arena_bytes, ci_basis** out, ci_stream stream)
{
    if (!probs || !info || n_probs <= 0) return fail(CI_EINVAL, "null pointer or n_probs <= 0");
    if (out) *out = nullptr;
    std::string err;
    // the plan of a size query with the same problems on this thread, else a new one
    std::unique_ptr<BuildPlan> P;
    if (t_pending && t_pending->keys == keys_of(probs, n_probs)) P = std::move(t_pending);
    t_pending.reset();
    if (!P) {
        P.reset(new BuildPlan());
        const int rc = plan_build(probs, n_probs, *P, err);
        if (rc != CI_OK) return fail(rc, err);
    }
    const std::vector<std::shared_ptr<HostBasis>>& ub = P->ub;
    if (!arena) {
        // size query: no device call; the table sizes follow the build
        int64_t R = 0;
        for (int32_t b = 0; b < n_probs; b++) {
            const HostBasis& hb = *ub[P->which[b]];
            fill_info(hb, info[b]);
            info[b].n_tbme = -1;
            info[b].row_ptr_offset = R;
            info[b].tbme_offset = -1;
            info[b].index_bytes = -1;
            info[b].arena_bytes = (int64_t)P->bytes;
            info[b].list_bytes = -1;
            R += hb.dim + 1;
        }
        t_pending = std::move(P);
        return CI_OK;
    }
    if (!out) return fail(CI_EINVAL, "null pointer");
    if (arena_bytes < P->bytes) {
        t_pending = std::move(P);  // a retry with a larger arena plans nothing again
        return fail(CI_ESPACE, "the arena needs " + std::to_string(t_pending->bytes) + " bytes");
    }
    hipStream_t s = (hipStream_t)stream;
    std::unique_ptr<ci_basis> h(new ci_basis());
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    h->arena = (char*)arena;
    h->arena_bytes = P->bytes;
    char* dev = h->arena;
    auto D = [&](size_t off) { return (void*)(dev + off); };
    const size_t host_bytes = P->host_bytes, pair_start = P->pair_start;

    // host mirror of the host-written tables (pinned staging), then the list
    // lengths read back later
    char* mirror = pinned_staging(host_bytes);
    if (!mirror) return fail(CI_EHIP, "hipHostMalloc(staging buffer)");
    auto put = [&](size_t off, const void* src, size_t n) {
        if (n) std::memcpy(mirror + off, src, n);
    };
    for (size_t u = 0; u < ub.size(); u++) {
        const HostBasis& hb = *ub[u];
        for (int sidx = 0; sidx < 2; sidx++) {
            if (P->canon[2 * u + sidx] != (int)(2 * u + sidx)) continue;
            const HostSpecies& sp = hb.sp[sidx];
            const SpOff& o = P->uo[u].sp[sidx];
            put(o.sd, sp.sd.data(), sp.sd.size() * 8);
            {
                const int64_t nsd = sp.nsd();
                uint64_t* Tw = (uint64_t*)(mirror + o.sdT);
                for (int64_t x = 0; x < nsd; x++)
                    for (int w = 0; w < hb.W; w++) Tw[(int64_t)w * nsd + x] = sp.sd[x * hb.W + w];
            }
            put(o.sd_key, sp.sd_key.data(), sp.sd_key.size() * 4);
            put(o.key_off, sp.key_off.data(), sp.key_off.size() * 4);
            put(o.key_nq, sp.key_nq.data(), sp.key_nq.size() * 4);
            put(o.key_m2, sp.key_m2.data(), sp.key_m2.size() * 4);
        }
        const UOff& U = P->uo[u];
        put(U.blk_kp, hb.blk_kp.data(), hb.blk_kp.size() * 4);
        put(U.blk_kn, hb.blk_kn.data(), hb.blk_kn.size() * 4);
        put(U.blk_off, hb.blk_off.data(), hb.blk_off.size() * 8);
        {
            BlockInfo* bk = (BlockInfo*)(mirror + U.blk);
            for (int k = 0; k < hb.nblk(); k++) {
                const HostSpecies& N = hb.sp[1];
                bk[k].kp = hb.blk_kp[k];
                bk[k].kn = hb.blk_kn[k];
                bk[k].row0 = (int32_t)hb.blk_off[k];
                bk[k].nkn = N.key_off[hb.blk_kn[k] + 1] - N.key_off[hb.blk_kn[k]];
            }
        }
        put(U.orb_n, hb.orb_n.data(), hb.orb_n.size() * 4);
        {
            int32_t* q = (int32_t*)(mirror + U.orb_qn);
            for (int o = 0; o < hb.nsps; o++)
                q[o] = ((hb.orb_n[o] - hb.orb_l[o]) / 2) | (hb.orb_l[o] << 8) | (hb.orb_j2[o] << 16) |
                       ((hb.orb_m2[o] + 64) << 24);
        }
    }
    std::vector<int64_t> first(n_probs), last(n_probs), row0(n_probs + 1, 0);
    int64_t R = 0;
    for (int32_t b = 0; b < n_probs; b++) {
        const HostBasis& hb = *ub[P->which[b]];
        first[b] = R;
        last[b] = R + hb.dim;
        row0[b + 1] = row0[b] + hb.dim;
        R += hb.dim + 1;
    }
    {
        int32_t* bb = (int32_t*)(mirror + P->o_blk_basis);
        int32_t* bl = (int32_t*)(mirror + P->o_blk_local);
        int gb = 0;
        for (int32_t b = 0; b < n_probs; b++)
            for (int k = 0; k < ub[P->which[b]]->nblk(); k++, gb++) {
                bb[gb] = b;
                bl[gb] = k;
            }
    }
    put(P->o_row0, row0.data(), row0.size() * 8);
    put(P->o_first, first.data(), first.size() * 8);
    put(P->o_last, last.data(), last.size() * 8);
    {
        std::vector<uint64_t*> outp(ub.size());
        for (size_t u = 0; u < ub.size(); u++) outp[u] = (uint64_t*)(mirror + P->uo[u].pair);
        P->pairs->set_targets(outp);
    }
    e = hipMemcpyAsync(dev, mirror, pair_start, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(index tables)");

    // what the partner lists need later
    h->uniq = ub;
    h->which = P->which;
    h->canon = P->canon;
    h->uo = P->uo;

    // ---- partner lists on the device: count and scan (the lengths are read
    // back by ci_basis_list_bytes)
    int64_t* scan_tmp = (int64_t*)D(P->o_scan);
    for (size_t u = 0; u < ub.size(); u++)
        for (int sidx = 0; sidx < 2; sidx++) {
            if (P->canon[2 * u + sidx] != (int)(2 * u + sidx)) continue;
            PartnerArgs a = partner_args(*h, u, sidx);
            if ((e = launch_partner_count(a, s)) != hipSuccess) return hip_fail(e, "partner count");
            // the count pass leaves l*_ptr[0] = 0; the inclusive scan gives offsets
            if ((e = launch_inclusive_scan(a.l1_ptr, a.nsd + 1, scan_tmp, s)) != hipSuccess ||
                (e = launch_inclusive_scan(a.l12_ptr, a.nsd + 1, scan_tmp, s)) != hipSuccess)
                return hip_fail(e, "partner scan");
            int64_t* tot = (int64_t*)D(P->uo[u].totals);
            if ((e = launch_copy_i64(a.l1_ptr + a.nsd, tot + 2 * sidx, s)) != hipSuccess ||
                (e = launch_copy_i64(a.l12_ptr + a.nsd, tot + 2 * sidx + 1, s)) != hipSuccess)
                return hip_fail(e, "partner totals");
        }
    // two-body pair indexes (helper thread) while the partner lists are counted
    {
        size_t bad = 0;
        const int rc = P->pairs->wait(&bad, err);
        if (rc != CI_OK) return fail(rc, "problem " + std::to_string(bad) + ": " + err);
    }
    // its upload (1.4 MB for 6Li Nmax = 6, tens of microseconds over PCIe)
    // overlaps the partner-list kernels; the stream waits for it before the
    // row kernels that read it
    e = copy_beside(dev + pair_start, mirror + pair_start, host_bytes - pair_start, s, h->device);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(pair index)");
    e = staging_fence(s, h->device);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord(staging)");

    // ---- per-problem descriptors (uploaded with the partner lists)
    h->bd.assign(n_probs, BasisDev{});
    R = 0;
    int64_t T = 0;
    h->info.resize(n_probs);
    for (int32_t b = 0; b < n_probs; b++) {
        const size_t u = (size_t)P->which[b];
        const HostBasis& hb = *ub[u];
        BasisDev& d = h->bd[b];
        std::memset(&d, 0, sizeof d);
        for (int sidx = 0; sidx < 2; sidx++) {
            const SpOff& o = P->uo[u].sp[sidx];
            SpeciesDev& sd = d.sp[sidx];
            sd.sd = (const uint64_t*)D(o.sd);
            sd.key_off = (const int32_t*)D(o.key_off);
            sd.l1_ptr = (const int64_t*)D(o.l1_ptr);
            sd.l12_ptr = (const int64_t*)D(o.l12_ptr);
            sd.seg1 = (const int32_t*)D(o.seg1);
            sd.seg12 = (const int32_t*)D(o.seg12);
            sd.self12 = (const int32_t*)D(o.self12);
            sd.nsd = (int32_t)hb.sp[sidx].nsd();
            sd.nk = hb.sp[sidx].nk();
        }
        const UOff& U = P->uo[u];
        d.blk_kp = (const int32_t*)D(U.blk_kp);
        d.blk_kn = (const int32_t*)D(U.blk_kn);
        d.blk_off = (const int64_t*)D(U.blk_off);
        d.blk = (const BlockInfo*)D(U.blk);
        d.pair = (const uint64_t*)D(U.pair);
        d.orb_n = (const int32_t*)D(U.orb_n);
        d.orb_qn = (const int32_t*)D(U.orb_qn);
        d.kinetic = hb.prob.kinetic;
        d.dim = hb.dim;
        d.row0 = R;
        d.tbme0 = T;
        d.ntbme = hb.n_tbme;
        d.W = hb.W;
        d.nsps = hb.nsps;
        d.nblk = hb.nblk();
        d.nsec = (int32_t)hb.sec_n.size();
        d.Z = hb.prob.Z;
        d.NN = hb.prob.N;
        d.hw = hb.prob.hw_mev;
        fill_info(hb, info[b]);
        info[b].row_ptr_offset = R;
        info[b].tbme_offset = T;
        info[b].index_bytes = -1;  // known once the lists are counted
        info[b].arena_bytes = (int64_t)P->bytes;
        info[b].list_bytes = -1;
        h->info[b] = info[b];
        h->host.push_back(ub[u]);
        R += hb.dim + 1;
        T += hb.n_tbme;
    }
    h->d_bases = (BasisDev*)D(P->o_bases);
    h->d_basis_row0 = (int64_t*)D(P->o_row0);
    h->d_seg_first = (int64_t*)D(P->o_first);
    h->d_seg_last = (int64_t*)D(P->o_last);
    h->d_scan_tmp = scan_tmp;
    h->d_nnz = (int64_t*)D(P->o_nnz);
    h->d_queue = (unsigned long long*)D(P->o_queue);
    h->d_rec_count = (unsigned long long*)D(P->o_rec_count);
    h->d_gscale = (unsigned long long*)D(P->o_gscale);
    h->d_blk_basis = (int32_t*)D(P->o_blk_basis);
    h->d_blk_local = (int32_t*)D(P->o_blk_local);
    h->d_tile_off = (int64_t*)D(P->o_tile_off);
    h->d_adjb = (AdjBasis*)D(P->o_adjb);
    h->nblocks = P->nblocks;
    h->probs.assign(probs, probs + n_probs);
    h->tune = cached_tuning(h->probs);
    h->nrows = row0[n_probs];
    h->n_rowptr = R;
    h->n_tbme = T;
    // the partner lists are still being counted on the stream
    *out = h.release();
    return CI_OK;
}

int ci_basis_list_bytes(ci_basis* b, size_t* bytes, ci_stream stream)
{
    if (!b || !bytes) return fail(CI_EINVAL, "null pointer");
    if (!b->lists_counted) {
        hipStream_t s = (hipStream_t)stream;
        const size_t nu = b->uniq.size();
        int64_t* pin = pinned_counts(4 * nu);
        if (!pin) return fail(CI_EHIP, "hipHostMalloc(counts)");
        for (size_t u = 0; u < nu; u++) {
            hipError_t e = hipMemcpyAsync(pin + 4 * u, b->arena + b->uo[u].totals, 4 * sizeof(int64_t),
                                          hipMemcpyDeviceToHost, s);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(list lengths)");
        }
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(partner count)");
        std::vector<int64_t> totals(pin, pin + 4 * nu);
        const int nsp = 2 * (int)nu;
        for (int i = 0; i < nsp; i++) {
            const int c = b->canon[i];
            totals[2 * i] = totals[2 * c];
            totals[2 * i + 1] = totals[2 * c + 1];
        }
        Layout LL;
        b->lo1.assign(nsp, 0);
        b->lo12.assign(nsp, 0);
        for (int i = 0; i < nsp; i++) {
            if (b->canon[i] != i) {
                b->lo1[i] = b->lo1[b->canon[i]];
                b->lo12[i] = b->lo12[b->canon[i]];
                continue;
            }
            b->lo1[i] = LL.take<uint64_t>(std::max<int64_t>(totals[2 * i], 1));
            b->lo12[i] = LL.take<uint64_t>(std::max<int64_t>(totals[2 * i + 1], 1));
        }
        b->totals = totals;
        b->list_bytes = LL.bytes();
        for (size_t p = 0; p < b->info.size(); p++) {
            const size_t u = (size_t)b->which[p];
            int64_t lb = 0;
            for (int sidx = 0; sidx < 2; sidx++) lb += 8 * (totals[4 * u + 2 * sidx] + totals[4 * u + 2 * sidx + 1]);
            b->info[p].index_bytes = (int64_t)b->uo[u].bytes + lb;
            b->info[p].list_bytes = (int64_t)b->list_bytes;
        }
        b->lists_counted = true;
    }
    *bytes = b->list_bytes;
    return CI_OK;
}

int ci_basis_build_lists(ci_basis* b, void* lists, size_t bytes, ci_stream stream)
{
    if (!b || !lists) return fail(CI_EINVAL, "null pointer");
    if (!b->lists_counted) return fail(CI_EINVAL, "the lists are not counted yet (ci_basis_list_bytes)");
    if (b->ready) return fail(CI_EINVAL, "the partner lists of this basis are already built");
    if (bytes < b->list_bytes)
        return fail(CI_ESPACE, "the partner lists need " + std::to_string(b->list_bytes) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    char* ldev = (char*)lists;
    hipError_t e = hipSuccess;
    for (size_t u = 0; u < b->uniq.size(); u++)
        for (int sidx = 0; sidx < 2; sidx++) {
            const int i = 2 * (int)u + sidx;
            if (b->canon[i] != i) continue;
            PartnerArgs a = partner_args(*b, u, sidx);
            a.l1 = (uint64_t*)(ldev + b->lo1[i]);
            a.l12 = (uint64_t*)(ldev + b->lo12[i]);
            if ((e = launch_partner_fill(a, b->totals[2 * i], b->totals[2 * i + 1], s)) != hipSuccess)
                return hip_fail(e, "partner fill");
        }
    // descriptors with the list pointers, one copy out of the staging buffer
    const size_t n = b->bd.size();
    for (size_t p = 0; p < n; p++) {
        const size_t u = (size_t)b->which[p];
        for (int sidx = 0; sidx < 2; sidx++) {
            const int i = 2 * (int)u + sidx;
            b->bd[p].sp[sidx].l1 = (const uint64_t*)(ldev + b->lo1[i]);
            b->bd[p].sp[sidx].l12 = (const uint64_t*)(ldev + b->lo12[i]);
        }
    }
    char* mirror = pinned_staging(n * sizeof(BasisDev));
    if (!mirror) return fail(CI_EHIP, "hipHostMalloc(staging buffer)");
    std::memcpy(mirror, b->bd.data(), n * sizeof(BasisDev));
    e = hipMemcpyAsync(b->d_bases, mirror, n * sizeof(BasisDev), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(descriptors)");
    e = staging_fence(s, b->device);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord(staging)");
    b->lists = ldev;
    b->ready = true;
    return CI_OK;
}

void ci_basis_free(ci_basis* b) { delete b; }


int32_t ci_basis_count(const ci_basis* b) { return b ? (int32_t)b->info.size() : 0; }

int ci_basis_get_info(const ci_basis* b, int32_t prob, ci_basis_info* info)
{
    if (!b || !info) return fail(CI_EINVAL, "null pointer");
    if (prob < 0 || prob >= (int32_t)b->info.size()) return fail(CI_EINVAL, "problem index out of range");
    *info = b->info[prob];
    return CI_OK;
}

static int count_impl(const ci_basis* b, int64_t* row_ptr, int64_t* nnz, int full, hipStream_t s)
{
    if (!b || !row_ptr || !nnz) return fail(CI_EINVAL, "null pointer");
    if (int rc = need_ready(b)) return rc;
    const int n = (int)b->info.size();
    hipError_t e = launch_count(b->d_bases, n, b->d_basis_row0, b->nrows, row_ptr, b->n_rowptr, b->d_seg_first,
                                b->d_scan_tmp, b->tune, b->d_queue, full, s);
    if (e != hipSuccess) return hip_fail(e, "count launch");
    e = launch_nnz(row_ptr, b->d_seg_first, b->d_seg_last, b->d_nnz, n, s);
    if (e != hipSuccess) return hip_fail(e, "nnz launch");
    int64_t* pin = pinned_counts(n);
    if (!pin) return fail(CI_EHIP, "hipHostMalloc(counts)");
    e = hipMemcpyAsync(pin, b->d_nnz, n * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(nnz)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(count)");
    std::memcpy(nnz, pin, n * sizeof(int64_t));
    if (!full) {
        int64_t tot = 0;
        for (int p = 0; p < n; p++) tot += nnz[p];
        b->nnz_total = tot;
    }
    return CI_OK;
}

static int fill_impl(const ci_basis* b, const float* tbme, const int64_t* row_ptr, int32_t* col, float* val,
                     uint32_t* keys, int full, hipStream_t s)
{
    if (!b || !row_ptr) return fail(CI_EINVAL, "null pointer");
    if (int rc = need_ready(b)) return rc;
    if (!tbme && b->n_tbme > 0) return fail(CI_EINVAL, "null pointer");
    hipError_t e = launch_fill(b->d_bases, (int)b->info.size(), b->d_basis_row0, b->nrows, tbme, row_ptr,
                               b->n_rowptr, col, val, keys, b->tune, b->d_queue, full, s);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    return CI_OK;
}

int ci_hamiltonian_count(const ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream)
{
    return count_impl(b, row_ptr, nnz, 0, (hipStream_t)stream);
}

int ci_hamiltonian_fill(const ci_basis* b, const float* tbme, const int64_t* row_ptr, int32_t* col,
                        float* val, ci_stream stream)
{
    return fill_impl(b, tbme, row_ptr, col, val, nullptr, 0, (hipStream_t)stream);
}

// The stored words hold a table position of the entry's basis in 30 bits.
static bool keys_fit(const ci_basis* b)
{
    for (const auto& i : b->info)
        if (i.n_tbme >= (int64_t)0x3fffffff) return false;
    return true;
}

int ci_hamiltonian_fill_keys(const ci_basis* b, const float* tbme, const int64_t* row_ptr, int32_t* col,
                             float* val, uint32_t* keys, ci_stream stream)
{
    if (!b) return fail(CI_EINVAL, "null pointer");
    if (!keys && b->nrows > 0) return fail(CI_EINVAL, "null pointer");
    if (!keys_fit(b)) return fail(CI_EUNSUPPORTED, "two-body table too large for the stored words");
    return fill_impl(b, tbme, row_ptr, col, val, keys, 0, (hipStream_t)stream);
}

int ci_hamiltonian_count_full(const ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream)
{
    return count_impl(b, row_ptr, nnz, 1, (hipStream_t)stream);
}

int ci_hamiltonian_fill_full(const ci_basis* b, const float* tbme, const int64_t* row_ptr, int32_t* col,
                             float* val, ci_stream stream)
{
    return fill_impl(b, tbme, row_ptr, col, val, nullptr, 1, (hipStream_t)stream);
}

static int h3_check(const ci_basis* b)
{
    for (const auto& p : b->probs)
        if (p.Z + p.N > 128) return fail(CI_EUNSUPPORTED, "the three-body term takes at most 128 nucleons");
    return CI_OK;
}

// The partner indexes of every basis, neutrons and protons (d <= 2 partners
// in every key):
// count, scan, read back the length, fill.  Synchronizes the stream once per
// basis, on the first three-body call of the handle.
static int h3_build_index(ci_basis* b, hipStream_t s)
{
    if (!b->h3_index.empty()) return CI_OK;
    const size_t n = b->host.size();
    std::vector<const void*> idx(6 * n, nullptr);
    std::vector<void*> mem;
    auto cleanup = [&]() {
        for (void* m : mem) (void)hipFree(m);
    };
    for (size_t p = 0; p < n; p++) {
        const HostBasis& hb = *b->host[p];
        for (int k = 0; k < 2; k++) {
            const int species = k == 0 ? 1 : 0;  // neutrons first, then protons
            const HostSpecies& S = hb.sp[species];
            const int64_t nsd = S.nsd();
            const size_t seg_bytes = ((size_t)nsd * (S.nk() + 1) * 4 + 255) / 256 * 256;
            const size_t ptr_bytes = ((size_t)(nsd + 1) * 8 + 255) / 256 * 256;
            void* head = nullptr;
            hipError_t e = hipMalloc(&head, seg_bytes + 2 * ptr_bytes);
            if (e != hipSuccess) return cleanup(), hip_fail(e, "hipMalloc(three-body index)");
            mem.push_back(head);
            int32_t* seg = (int32_t*)head;
            int64_t* ptr = (int64_t*)((char*)head + seg_bytes);
            int64_t* tmp = (int64_t*)((char*)head + seg_bytes + ptr_bytes);
            int64_t total = 0;
            if (nsd > 0) {  // (with no determinant the basis has no row to read the index)
                e = launch_h3_index(false, b->d_bases + p, species, nsd, hb.W, seg, ptr, nullptr, s);
                if (e == hipSuccess) e = launch_inclusive_scan(ptr, nsd + 1, tmp, s);
                if (e == hipSuccess) e = hipMemcpyAsync(&total, ptr + nsd, sizeof(int64_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
            }
            if (e != hipSuccess) return cleanup(), hip_fail(e, "three-body index count");
            void* rec = nullptr;
            e = hipMalloc(&rec, (size_t)std::max<int64_t>(total, 1) * 8);
            if (e != hipSuccess) return cleanup(), hip_fail(e, "hipMalloc(three-body index records)");
            mem.push_back(rec);
            if (nsd > 0) e = launch_h3_index(true, b->d_bases + p, species, nsd, hb.W, seg, ptr, (uint64_t*)rec, s);
            if (e != hipSuccess) return cleanup(), hip_fail(e, "three-body index fill");
            idx[6 * p + 3 * k] = seg;
            idx[6 * p + 3 * k + 1] = ptr;
            idx[6 * p + 3 * k + 2] = rec;
        }
    }
    b->h3_index = idx;
    b->h3_mem = mem;
    return CI_OK;
}

static std::vector<int64_t> h3_dims(const ci_basis* b)
{
    std::vector<int64_t> d(b->info.size());
    for (size_t p = 0; p < d.size(); p++) d[p] = b->info[p].dim;
    return d;
}

static std::vector<int> h3_words(const ci_basis* b)
{
    std::vector<int> w(b->host.size());
    for (size_t p = 0; p < w.size(); p++) w[p] = b->host[p]->W;
    return w;
}

static int h3_count_impl(ci_basis* b, int64_t* row_ptr, int64_t* nnz, int full, ci_stream stream)
{
    if (!b || !row_ptr || !nnz) return fail(CI_EINVAL, "null pointer");
    if (int rc = need_ready(b)) return rc;
    if (int rc = h3_check(b)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (int rc = h3_build_index(b, s)) return rc;
    const int n = (int)b->info.size();
    const std::vector<int64_t> dims = h3_dims(b);
    const std::vector<int> words = h3_words(b);
    hipError_t e = launch_h3_rows(b->d_bases, dims.data(), words.data(), b->h3_index.data(), n, nullptr, 0, 0, 0.0,
                                  row_ptr, nullptr, nullptr, false, full, s);
    if (e != hipSuccess) return hip_fail(e, "three-body count launch");
    e = launch_inclusive_scan(row_ptr, b->n_rowptr, b->d_scan_tmp, s);
    if (e != hipSuccess) return hip_fail(e, "scan launch");
    e = launch_nnz(row_ptr, b->d_seg_first, b->d_seg_last, b->d_nnz, n, s);
    if (e != hipSuccess) return hip_fail(e, "nnz launch");
    int64_t* pin = pinned_counts(n);
    if (!pin) return fail(CI_EHIP, "hipHostMalloc(counts)");
    e = hipMemcpyAsync(pin, b->d_nnz, n * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(nnz)");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(three-body count)");
    std::memcpy(nnz, pin, n * sizeof(int64_t));
    return CI_OK;
}

static int h3_fill_impl(ci_basis* b, const float* tbme, const ci_v3* v3, const int64_t* row_ptr, int32_t* col,
                        float* val, int full, ci_stream stream)
{
    if (!b || !v3 || !row_ptr) return fail(CI_EINVAL, "null pointer");
    if (v3->kind < CI_V3_NONE || v3->kind > CI_V3_IDENTITY) return fail(CI_EINVAL, "unknown three-body kind");
    if (int rc = need_ready(b)) return rc;
    if (!tbme && b->n_tbme > 0) return fail(CI_EINVAL, "null pointer");
    if (int rc = h3_check(b)) return rc;
    if (int rc = h3_build_index(b, (hipStream_t)stream)) return rc;
    const std::vector<int64_t> dims = h3_dims(b);
    const std::vector<int> words = h3_words(b);
    hipError_t e = launch_h3_rows(b->d_bases, dims.data(), words.data(), b->h3_index.data(), (int)dims.size(), tbme,
                                  v3->kind, v3->seed, v3->scale, const_cast<int64_t*>(row_ptr), col, val, true, full,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "three-body fill launch");
    return CI_OK;
}

int ci_hamiltonian3_count(ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream)
{
    return h3_count_impl(b, row_ptr, nnz, 0, stream);
}

int ci_hamiltonian3_fill(ci_basis* b, const float* tbme, const ci_v3* v3, const int64_t* row_ptr, int32_t* col,
                         float* val, ci_stream stream)
{
    return h3_fill_impl(b, tbme, v3, row_ptr, col, val, 0, stream);
}

int ci_hamiltonian3_count_full(ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream)
{
    return h3_count_impl(b, row_ptr, nnz, 1, stream);
}

int ci_hamiltonian3_fill_full(ci_basis* b, const float* tbme, const ci_v3* v3, const int64_t* row_ptr, int32_t* col,
                              float* val, ci_stream stream)
{
    return h3_fill_impl(b, tbme, v3, row_ptr, col, val, 1, stream);
}

// Adjoint tiles of basis p for shape t (the device computes the same counts
// in tile_offsets).
static int64_t count_tiles_of(const HostBasis& hb, const ci_tuning& t, bool stored)
{
    const int64_t rows = stored ? t.adjk_rows : t.adj_rows, tile_n = stored ? t.adjk_tile_n : t.adj_tile_n;
    int64_t n = 0;
    for (int bi = 0; bi < hb.nblk(); bi++) {
        const HostSpecies &P = hb.sp[0], &N = hb.sp[1];
        const int64_t nKp = P.key_off[hb.blk_kp[bi] + 1] - P.key_off[hb.blk_kp[bi]];
        const int64_t nKn = N.key_off[hb.blk_kn[bi] + 1] - N.key_off[hb.blk_kn[bi]];
        const int64_t tn = std::min<int64_t>(tile_n, nKn);
        const int64_t tp = std::max<int64_t>(1, rows / tn);
        n += ((nKp + tp - 1) / tp) * ((nKn + tn - 1) / tn);
    }
    return n;
}

// Work buffer of one adjoint launch: int64 fixed-point accumulators of the
// contributions that find no table slot (or no room in the record buffer)
// [n_tbme], the tile records (uint64: table position | int32 fixed-point tile
// sum << 32), the bucket-major
// histograms (int32 record positions, one per tile and bucket).  The record buffer holds at most as many
// records as the tiles have slots, and no more than half the stored entries
// (a tile writes one record per distinct table position it touched: about a
// quarter to a third of the entries at the tuned shapes; a tile that finds
// no room adds its sums to the accumulators instead).
// Without records (histograms beyond kHistCap entries: tiny tiles) the tiles
// add their sums to the accumulators directly.
constexpr int64_t kHistCap = (int64_t)1 << 25;

struct VjpLayout {
    int64_t ntiles = 0, nbuckets = 0, rec_cap = 0;
    int chunks = 1;  // tile chunks per bucket in the reduction (> 1: int64 partial sums at part)
    bool records = false;
    size_t recs = 0, hist = 0, part = 0, bytes = 0;
};

// The reduction runs one workgroup per (bucket, chunk of tiles); with few
// buckets the tiles are cut into chunks so that about 512 workgroups share the
// work, each chunk's int64 partial sums taking n_tbme words (at most 256 MiB).
static int reduce_chunks(int64_t nbuckets, int64_t n_tbme)
{
    int c = (int)std::min<int64_t>(kAdjMaxChunks, std::max<int64_t>(1, 512 / std::max<int64_t>(nbuckets, 1)));
    while (c > 1 && (int64_t)c * n_tbme * (int64_t)sizeof(int64_t) > ((int64_t)256 << 20)) c--;
    return c;
}

static VjpLayout vjp_layout(const ci_basis* b, const ci_tuning& t, bool stored, size_t limit = 0)
{
    VjpLayout v;
    int64_t hist = 0;
    for (size_t p = 0; p < b->host.size(); p++) {
        const int64_t nt = count_tiles_of(*b->host[p], t, stored);
        const int nb = adj_buckets(b->info[p].n_tbme);
        v.ntiles += nt;
        v.nbuckets += nb;
        hist += nt * (nb + 1);
    }
    v.records = t.adj_flush == 0 && hist <= kHistCap && b->n_tbme < 0xffffffffLL;
    Layout L;
    (void)L.take<int64_t>((size_t)b->n_tbme);
    if (v.records) {
        v.rec_cap = v.ntiles * (int64_t)adjoint_slots(stored || t.adj_wide);
        if (b->nnz_total >= 0) v.rec_cap = std::min<int64_t>(v.rec_cap, b->nnz_total / 2 + 1);
        v.rec_cap = std::min<int64_t>(v.rec_cap, INT32_MAX);  // record positions are int32 in the histograms
        v.hist = L.take<int32_t>((size_t)std::max<int64_t>(hist, 1));
        v.chunks = reduce_chunks(v.nbuckets, b->n_tbme);
        if (limit && L.bytes() + (size_t)v.chunks * b->n_tbme * sizeof(int64_t) + 4096 > limit) v.chunks = 1;
        if (v.chunks > 1) v.part = L.take<int64_t>((size_t)v.chunks * b->n_tbme);
        if (limit) {  // a fixed buffer: the records get what is left of it
            const size_t left = limit > L.bytes() + 256 ? limit - L.bytes() - 256 : 0;
            v.rec_cap = std::min<int64_t>(v.rec_cap, (int64_t)(left / sizeof(uint64_t)));
            if (v.rec_cap < 1 || L.bytes() > limit) v.records = false;
        }
        v.recs = L.take<uint64_t>((size_t)std::max<int64_t>(v.rec_cap, 1));
    }
    if (!v.records) {
        v.rec_cap = 0;
        v.chunks = 1;
        v.recs = v.hist = v.part = 0;
        L = Layout();
        (void)L.take<int64_t>((size_t)b->n_tbme);
    }
    v.bytes = L.bytes();
    return v;
}

// Launch shapes the autotuner tries for the adjoint (tile rows, neutron width).
// walking adjoint: (rows, neutron width, wide table)
static const int kWalkTiles[][3] = {{32, 8, 0},   {64, 8, 0},   {64, 16, 0},  {128, 16, 0}, {64, 16, 1},
                                    {96, 16, 1},  {128, 16, 1}, {192, 16, 1}, {256, 16, 1}, {256, 32, 1},
                                    {512, 32, 1}};
static const int kStoredTiles[][2] = {{64, 8}, {96, 8}, {128, 8}, {96, 16}, {192, 8}, {256, 16}};

static size_t work_bytes_for(const ci_basis* b)
{
    size_t w = std::max(vjp_layout(b, b->tune, false).bytes, vjp_layout(b, b->tune, true).bytes);
    ci_tuning t = b->tune;
    t.adj_flush = 0;  // the records need the larger buffer
    w = std::max(w, std::max(vjp_layout(b, t, false).bytes, vjp_layout(b, t, true).bytes));
    for (const auto& tl : kWalkTiles) {
        t.adj_rows = tl[0];
        t.adj_tile_n = tl[1];
        t.adj_wide = tl[2];
        w = std::max(w, vjp_layout(b, t, false).bytes);
    }
    t = b->tune;
    t.adj_flush = 0;
    for (const auto& tl : kStoredTiles) {
        t.adjk_rows = tl[0];
        t.adjk_tile_n = tl[1];
        w = std::max(w, vjp_layout(b, t, true).bytes);
    }
    return w;
}

static hipError_t vjp_launch(const ci_basis* b, const int64_t* row_ptr, const float* grad_val, float* grad_tbme,
                             void* work, const ci_tuning& t, hipStream_t s, const uint32_t* keys = nullptr,
                             size_t limit = 0)
{
    const bool stored = keys != nullptr;
    const VjpLayout v = vjp_layout(b, t, stored, limit);
    char* w = (char*)work;
    ci_tuning tt = t;
    if (stored) tt.adj_persistent = t.adjk_persistent;
    return launch_vjp(b->d_bases, (int)b->info.size(), b->d_blk_basis, b->d_blk_local, b->nblocks, v.ntiles,
                      b->d_tile_off, b->d_adjb, v.nbuckets, v.chunks,
                      v.chunks > 1 ? (unsigned long long*)(w + v.part) : nullptr, b->nrows, row_ptr, b->n_rowptr,
                      grad_val, keys, grad_tbme, (unsigned long long*)w,
                      v.records ? (uint64_t*)(w + v.recs) : nullptr, v.rec_cap, b->d_rec_count,
                      v.records ? (int32_t*)(w + v.hist) : nullptr, b->n_tbme, tt, b->d_queue, b->d_gscale,
                      b->nnz_total, s);
}

size_t ci_vjp_work_bytes(const ci_basis* b) { return (b && b->ready) ? work_bytes_for(b) : 0; }

int ci_hamiltonian_vjp(const ci_basis* b, const int64_t* row_ptr, const float* grad_val, float* grad_tbme,
                       void* work, size_t work_bytes, ci_stream stream)
{
    // every row stores its diagonal, so grad_val may be null only without rows
    if (!b || !row_ptr) return fail(CI_EINVAL, "null pointer");
    if (int rc = need_ready(b)) return rc;
    if (!grad_val && b->nrows > 0) return fail(CI_EINVAL, "null pointer");
    if (b->n_tbme > 0 && (!grad_tbme || !work)) return fail(CI_EINVAL, "null pointer");
    if (work_bytes < ci_vjp_work_bytes(b))
        return fail(CI_ESPACE, "vjp work buffer needs " + std::to_string(ci_vjp_work_bytes(b)) + " bytes");
    hipError_t e = vjp_launch(b, row_ptr, grad_val, grad_tbme, work, b->tune, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "vjp launch");
    return CI_OK;
}

int ci_hamiltonian_vjp_keys(const ci_basis* b, const int64_t* row_ptr, const uint32_t* keys, const float* grad_val,
                            float* grad_tbme, void* work, size_t work_bytes, ci_stream stream)
{
    if (!b || !row_ptr) return fail(CI_EINVAL, "null pointer");
    if (int rc = need_ready(b)) return rc;
    if ((!grad_val || !keys) && b->nrows > 0) return fail(CI_EINVAL, "null pointer");
    if (b->n_tbme > 0 && (!grad_tbme || !work)) return fail(CI_EINVAL, "null pointer");
    if (!keys_fit(b)) return fail(CI_EUNSUPPORTED, "two-body table too large for the stored words");
    if (work_bytes < ci_vjp_work_bytes(b))
        return fail(CI_ESPACE, "vjp work buffer needs " + std::to_string(ci_vjp_work_bytes(b)) + " bytes");
    hipError_t e = vjp_launch(b, row_ptr, grad_val, grad_tbme, work, b->tune, (hipStream_t)stream, keys);
    if (e != hipSuccess) return hip_fail(e, "vjp launch");
    return CI_OK;
}

int ci_hamiltonian_vjp_noalloc(const ci_basis* b, const int64_t* row_ptr, const float* grad_val, float* grad_tbme,
                               ci_stream stream)
{
    if (!b || !row_ptr) return fail(CI_EINVAL, "null pointer");
    if (int rc = need_ready(b)) return rc;
    if (!grad_val && b->nrows > 0) return fail(CI_EINVAL, "null pointer");
    if (b->n_tbme > 0 && !grad_tbme) return fail(CI_EINVAL, "null pointer");
    const size_t cap = noalloc_scratch_bytes();
    // the int64 accumulators must fit; the tile records take what is left
    if ((size_t)b->n_tbme * sizeof(int64_t) + 256 > cap)
        return fail(CI_ESPACE, "the two-body tables of this handle (" + std::to_string(b->n_tbme) +
                                   " elements) exceed the fixed scratch of " + std::to_string(cap) + " bytes");
    void* scr = nullptr;
    hipError_t e = noalloc_scratch(&scr);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    e = vjp_launch(b, row_ptr, grad_val, grad_tbme, scr, b->tune, (hipStream_t)stream, nullptr, cap);
    if (e != hipSuccess) return hip_fail(e, "vjp launch");
    return CI_OK;
}

size_t ci_vjp_noalloc_scratch_bytes(void) { return noalloc_scratch_bytes(); }

static bool tuning_ok(const ci_tuning& t)
{
    return (t.row_waves == 4 || t.row_waves == 8) && t.row_grab >= 0 && t.row_grab <= 4096 && t.adj_rows >= 1 &&
           t.adj_rows <= 4096 && t.adj_tile_n >= 1 && t.adj_tile_n <= 4096 &&
           (t.adj_persistent == 0 || t.adj_persistent == 1) && t.adjk_rows >= 1 && t.adjk_rows <= 4096 &&
           t.adjk_tile_n >= 1 && t.adjk_tile_n <= 4096 && (t.adjk_persistent == 0 || t.adjk_persistent == 1) &&
           (t.row_xcd == 0 || t.row_xcd == 1) && (t.adj_wide == 0 || t.adj_wide == 1) &&
           (t.adj_flush == 0 || t.adj_flush == 1);
}

int ci_basis_get_tuning(const ci_basis* b, ci_tuning* t)
{
    if (!b || !t) return fail(CI_EINVAL, "null pointer");
    *t = b->tune;
    return CI_OK;
}

int ci_basis_set_tuning(ci_basis* b, const ci_tuning* t)
{
    if (!b || !t) return fail(CI_EINVAL, "null pointer");
    if (!tuning_ok(*t)) return fail(CI_EINVAL, "launch shape out of range");
    b->tune = *t;
    return CI_OK;
}


int ci_hamiltonian_tune(ci_basis* b, const float* tbme, const int64_t* row_ptr, int32_t* col, float* val,
                        uint32_t* keys, const float* grad_val, float* grad_tbme, void* work, size_t work_bytes,
                        int32_t reps, ci_stream stream)
{
    if (!b || !row_ptr || !grad_val) return fail(CI_EINVAL, "null pointer");
    if (int rc = need_ready(b)) return rc;
    if (!tbme && b->n_tbme > 0) return fail(CI_EINVAL, "null pointer");
    if (b->n_tbme > 0 && (!grad_tbme || !work)) return fail(CI_EINVAL, "null pointer");
    if (reps < 1) return fail(CI_EINVAL, "reps must be >= 1");
    if (keys && !keys_fit(b)) return fail(CI_EUNSUPPORTED, "two-body table too large for the stored words");
    if (work_bytes < ci_vjp_work_bytes(b))
        return fail(CI_ESPACE, "vjp work buffer needs " + std::to_string(ci_vjp_work_bytes(b)) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    const ci_tuning start = b->tune;
    ci_tuning best = start;
    int rc = CI_OK;
    // fill: waves per workgroup x (grid, persistent with several grab sizes)
    float best_ms = 0.0f;
    bool have = false;
    for (int waves : {4, 8})
        for (int grab : {-1, 0, 1, 4, 16}) {  // -1: grid in XCD-contiguous order
            if (rc != CI_OK) break;
            b->tune = start;
            b->tune.row_waves = waves;
            b->tune.row_grab = grab < 0 ? 0 : grab;
            b->tune.row_xcd = grab < 0 ? 1 : 0;
            float ms = 0.0f;
            rc = time_ms([&] { return launch_fill(b->d_bases, (int)b->info.size(), b->d_basis_row0, b->nrows, tbme,
                                                  row_ptr, b->n_rowptr, col, val, nullptr, b->tune, b->d_queue, 0,
                                                  s); },
                         reps, s, e0, e1, &ms);
            if (rc == CI_OK && (!have || ms < best_ms)) {
                best_ms = ms;
                best.row_waves = waves;
                best.row_grab = b->tune.row_grab;
                best.row_xcd = b->tune.row_xcd;
                have = true;
            }
        }
    // adjoint that walks the partner lists: tile (rows, neutron width) x (grid, persistent)
    have = false;
    for (const auto& tl : kWalkTiles)
        for (int pers : {0, 1})
            for (int flush : {0, 1}) {
                if (rc != CI_OK) break;
                b->tune = best;
                b->tune.adj_rows = tl[0];
                b->tune.adj_tile_n = tl[1];
                b->tune.adj_wide = tl[2];
                b->tune.adj_persistent = pers;
                b->tune.adj_flush = flush;
                float ms = 0.0f;
                rc = time_ms([&] { return vjp_launch(b, row_ptr, grad_val, grad_tbme, work, b->tune, s); }, reps, s, e0,
                             e1, &ms);
                if (rc == CI_OK && (!have || ms < best_ms)) {
                    best_ms = ms;
                    best.adj_rows = tl[0];
                    best.adj_tile_n = tl[1];
                    best.adj_wide = tl[2];
                    best.adj_persistent = pers;
                    best.adj_flush = flush;
                    have = true;
                }
            }
    // adjoint from stored words (when the caller gives room for them): the
    // fill writes the words once, then its own tiles x (grid, persistent)
    if (keys && rc == CI_OK) {
        b->tune = best;
        e = launch_fill(b->d_bases, (int)b->info.size(), b->d_basis_row0, b->nrows, tbme, row_ptr, b->n_rowptr, col,
                        val, keys, b->tune, b->d_queue, 0, s);
        if (e != hipSuccess) rc = hip_fail(e, "autotune fill with stored words");
        have = false;
        for (const auto& tl : kStoredTiles)
            for (int pers : {0, 1}) {
                if (rc != CI_OK) break;
                b->tune = best;
                b->tune.adjk_rows = tl[0];
                b->tune.adjk_tile_n = tl[1];
                b->tune.adjk_persistent = pers;
                float ms = 0.0f;
                rc = time_ms([&] { return vjp_launch(b, row_ptr, grad_val, grad_tbme, work, b->tune, s, keys); }, reps,
                             s, e0, e1, &ms);
                if (rc == CI_OK && (!have || ms < best_ms)) {
                    best_ms = ms;
                    best.adjk_rows = tl[0];
                    best.adjk_tile_n = tl[1];
                    best.adjk_persistent = pers;
                    have = true;
                }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != CI_OK) {
        b->tune = start;
        return rc;
    }
    b->tune = best;
    remember_tuning(b->probs, best);
    // leave col / val (/ keys) / grad_tbme as the chosen shapes compute them
    e = launch_fill(b->d_bases, (int)b->info.size(), b->d_basis_row0, b->nrows, tbme, row_ptr, b->n_rowptr, col,
                    val, keys, b->tune, b->d_queue, 0, s);
    if (e == hipSuccess) e = vjp_launch(b, row_ptr, grad_val, grad_tbme, work, b->tune, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "autotune final run");
    return CI_OK;
}

static int spmv_any(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col, const float* val,
                    const double* x, double* y, ci_stream stream, bool upper)
{
    if (!b || !row_ptr || !x || !y) return fail(CI_EINVAL, "null pointer");
    if (prob < 0 || prob >= (int32_t)b->info.size()) return fail(CI_EINVAL, "problem index out of range");
    const ci_basis_info& I = b->info[prob];
    if (I.dim > 0 && (!col || !val)) return fail(CI_EINVAL, "null pointer");
    hipError_t e = upper ? launch_spmv_upper(row_ptr + I.row_ptr_offset, col, val, x, y, I.dim, (hipStream_t)stream)
                         : launch_spmv(row_ptr + I.row_ptr_offset, col, val, x, y, I.dim, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "spmv launch");
    return CI_OK;
}

int ci_hamiltonian_spmv(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col,
                        const float* val, const double* x, double* y, ci_stream stream)
{
    return spmv_any(b, prob, row_ptr, col, val, x, y, stream, false);
}

int ci_hamiltonian_spmv_upper(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col,
                              const float* val, const double* x, double* y, ci_stream stream)
{
    return spmv_any(b, prob, row_ptr, col, val, x, y, stream, true);
}

size_t ci_lanczos_work_bytes(int64_t dim, int32_t max_iter)
{
    return (dim > 0 && max_iter > 0) ? lanczos_work_bytes(dim, max_iter) : 0;
}

static int lanczos_any(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col, const float* val,
                       const double* x0, int32_t max_iter, double tol, double* eval, int32_t* iters, double* evec,
                       void* work, size_t work_bytes, ci_stream stream, bool upper)
{
    if (!b || !row_ptr || !col || !val || !x0 || !eval || !iters || !evec || !work)
        return fail(CI_EINVAL, "null pointer");
    if (prob < 0 || prob >= (int32_t)b->info.size()) return fail(CI_EINVAL, "problem index out of range");
    if (max_iter < 1 || max_iter > 4096 || !(tol >= 0.0)) return fail(CI_EINVAL, "max_iter in 1..4096, tol >= 0");
    const ci_basis_info& I = b->info[prob];
    if (I.dim < 1) return fail(CI_EINVAL, "empty basis");
    if (work_bytes < lanczos_work_bytes(I.dim, max_iter))
        return fail(CI_ESPACE, "Lanczos work buffer needs " + std::to_string(lanczos_work_bytes(I.dim, max_iter)) +
                                   " bytes");
    int it = 0;
    hipError_t e = run_lanczos(row_ptr + I.row_ptr_offset, col, val, I.dim, x0, max_iter, tol, eval, &it, evec, work,
                               (hipStream_t)stream, upper);
    if (e == hipErrorInvalidValue) return fail(CI_EINVAL, "start vector is zero");
    if (e != hipSuccess) return hip_fail(e, "lanczos");
    *iters = it;
    return CI_OK;
}

int ci_lanczos(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col, const float* val,
               const double* x0, int32_t max_iter, double tol, double* eval, int32_t* iters, double* evec,
               void* work, size_t work_bytes, ci_stream stream)
{
    return lanczos_any(b, prob, row_ptr, col, val, x0, max_iter, tol, eval, iters, evec, work, work_bytes, stream,
                       false);
}

int ci_lanczos_upper(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col, const float* val,
                     const double* x0, int32_t max_iter, double tol, double* eval, int32_t* iters, double* evec,
                     void* work, size_t work_bytes, ci_stream stream)
{
    return lanczos_any(b, prob, row_ptr, col, val, x0, max_iter, tol, eval, iters, evec, work, work_bytes, stream,
                       true);
}

struct ci_threebody {
    ThreeBodyHost h;
    ~ci_threebody() { threebody_release(h); }
};

int ci_threebody_plan(int32_t n1max, int32_t n3max, int64_t* n_coupled, int32_t* n_triples)
{
    if (!n_coupled || !n_triples) return fail(CI_EINVAL, "null pointer");
    ThreeBodyHost h;
    std::string err;
    const int rc = threebody_plan(n1max, n3max, h, err);
    if (rc != CI_OK) return fail(rc, err);
    *n_coupled = h.n_coupled;
    *n_triples = (int32_t)(h.trip.size() / 3);
    return CI_OK;
}

int ci_threebody_build(int32_t n1max, int32_t n3max, ci_threebody** out)
{
    if (!out) return fail(CI_EINVAL, "null pointer");
    *out = nullptr;
    std::unique_ptr<ci_threebody> t(new ci_threebody());
    std::string err;
    const int rc = threebody_plan(n1max, n3max, t->h, err);
    if (rc != CI_OK) return fail(rc, err);
    hipError_t e = threebody_upload(t->h);
    if (e != hipSuccess) return hip_fail(e, "three-body tables");
    *out = t.release();
    return CI_OK;
}

void ci_threebody_free(ci_threebody* t) { delete t; }

int ci_threebody_info(const ci_threebody* t, int64_t* n_coupled, int32_t* n_sps, int32_t* n_nlj, int32_t* n_triples)
{
    if (!t || !n_coupled || !n_sps || !n_nlj || !n_triples) return fail(CI_EINVAL, "null pointer");
    *n_coupled = t->h.n_coupled;
    *n_sps = (int32_t)t->h.orb_alpha.size();
    *n_nlj = (int32_t)t->h.nlj_j2.size();
    *n_triples = (int32_t)(t->h.trip.size() / 3);
    return CI_OK;
}

int ci_threebody_keys(const ci_threebody* t, int32_t* keys, int64_t cap)
{
    if (!t || (!keys && cap > 0)) return fail(CI_EINVAL, "null pointer");
    if (cap < t->h.n_coupled) return fail(CI_ESPACE, "need room for " + std::to_string(t->h.n_coupled) + " keys");
    threebody_keys(t->h, keys);
    return CI_OK;
}

int ci_threebody_orbitals(const ci_threebody* t, int32_t* nlj, int32_t* morb, int32_t* triples)
{
    if (!t || !nlj || !morb || !triples) return fail(CI_EINVAL, "null pointer");
    const ThreeBodyHost& h = t->h;
    for (size_t a = 0; a < h.nlj_j2.size(); a++) {
        nlj[3 * a] = h.nlj_N[a];
        nlj[3 * a + 1] = h.nlj_l[a];
        nlj[3 * a + 2] = h.nlj_j2[a];
    }
    for (size_t o = 0; o < h.orb_alpha.size(); o++) {
        morb[2 * o] = h.orb_alpha[o];
        morb[2 * o + 1] = h.orb_m2[o];
    }
    std::memcpy(triples, h.trip.data(), h.trip.size() * sizeof(int32_t));
    return CI_OK;
}

int ci_clebsch_gordan(int32_t j1, int32_t m1, int32_t j2, int32_t m2, int32_t J, int32_t M, double* out)
{
    if (!out) return fail(CI_EINVAL, "null pointer");
    if (j1 < 0 || j2 < 0 || J < 0 || j1 > 120 || j2 > 120 || J > 120)
        return fail(CI_EINVAL, "angular momenta (doubled) must lie in [0, 120]");
    *out = clebsch_gordan2(j1, m1, j2, m2, J, M);
    return CI_OK;
}

size_t ci_threebody_work_bytes(int64_t n) { return decouple_work_bytes(n); }

int ci_threebody_decouple(const ci_threebody* t, const float* coupled, const int32_t* requests, int64_t n,
                          float* out, void* work, size_t work_bytes, ci_stream stream)
{
    if (!t || n < 0 || (n > 0 && (!coupled || !requests || !out))) return fail(CI_EINVAL, "null pointer");
    if (work && n > 0x7fffffffLL) return fail(CI_EINVAL, "the cost order takes at most 2^31 - 1 requests");
    if (work && work_bytes < decouple_work_bytes(n))
        return fail(CI_ESPACE, "work needs " + std::to_string(decouple_work_bytes(n)) + " bytes");
    hipError_t e = launch_decouple(t->h, coupled, requests, n, work, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "decouple launch");
    return CI_OK;
}

int ci_probe_ceilings(void* buf, size_t bytes, double* store_gbs, double* diff_steps_per_s, ci_stream stream)
{
    if (!buf || !store_gbs || !diff_steps_per_s) return fail(CI_EINVAL, "null pointer");
    if (bytes < ((size_t)64 << 20)) return fail(CI_ESPACE, "the probe buffer needs at least 64 MiB");
    double bps = 0.0, steps = 0.0;
    hipError_t e = run_probes(buf, bytes, (hipStream_t)stream, &bps, &steps);
    if (e != hipSuccess) return hip_fail(e, "probe");
    *store_gbs = bps / 1e9;
    *diff_steps_per_s = steps;
    return CI_OK;
}

int ci_basis_states(const ci_basis* b, int32_t prob, uint64_t* bits, ci_stream stream)
{
    if (!b || !bits) return fail(CI_EINVAL, "null pointer");
    if (prob < 0 || prob >= (int32_t)b->info.size()) return fail(CI_EINVAL, "problem index out of range");
    const HostBasis& hb = *b->host[prob];
    const int W = hb.W;
    std::vector<uint64_t> st((size_t)hb.dim * 2 * W);
    int64_t i = 0;
    for (int bk = 0; bk < hb.nblk(); bk++) {
        const HostSpecies& P = hb.sp[0];
        const HostSpecies& N = hb.sp[1];
        for (int64_t p = P.key_off[hb.blk_kp[bk]]; p < P.key_off[hb.blk_kp[bk] + 1]; p++)
            for (int64_t q = N.key_off[hb.blk_kn[bk]]; q < N.key_off[hb.blk_kn[bk] + 1]; q++, i++) {
                std::memcpy(&st[(size_t)i * 2 * W], &P.sd[p * W], W * 8);
                std::memcpy(&st[(size_t)i * 2 * W + W], &N.sd[q * W], W * 8);
            }
    }
    hipError_t e = hipMemcpyAsync(bits, st.data(), st.size() * 8, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(states)");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(states)");
    return CI_OK;
}

}  // extern "C"
