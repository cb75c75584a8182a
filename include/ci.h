/*
 * ci.h -- C ABI of libci: construction of the sparse M-scheme many-body
 * Hamiltonian of a Configuration Interaction / No-Core Shell Model calculation
 * with a two-body interaction, on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the construction stage
 * (Potter et al., "Accelerating Ab Initio Nuclear Physics Calculations with
 * GPUs"):
 *   - Sec. 2: the indexing systems of the many-body basis are set up first
 *     (ci_basis_build); the symmetric matrix is generated and only half of it
 *     is stored; each element is a linear combination of one-body (kinetic /
 *     single-particle) and two-body interaction terms;
 *   - Sec. 4.1: the matrix is split into chunks of similar quantum numbers; the
 *     nonzeros are located twice, once to count them so that the arrays can be
 *     allocated (ci_hamiltonian_count) and once to calculate and store them
 *     (ci_hamiltonian_fill), in compressed-row (CSR) form;
 *   - Sec. 5.2: all index tables are built contiguously on the host and moved
 *     to the device in one allocation and one copy.
 * ci_hamiltonian_vjp is the adjoint of the fill with respect to the two-body
 * table (not in the paper).
 *
 * Conventions (the paper does not fix them; these are the textbook readings):
 *   orbits   harmonic-oscillator m-states of shells 0..S, S = max(Ntop(Z),
 *            Ntop(N)) + Nmax, ordered by N, l, 2j, 2m (ascending), the same
 *            set for both species.  Single-particle energy (N + 3/2) hw.
 *            Combined index: proton orbit k -> k, neutron orbit k -> n_sps + k.
 *   basis    proton and neutron Slater determinants as n_words 64-bit words
 *            (orbit k -> word k/64, bit k%64); a state is kept if its total
 *            oscillator quanta Nq <= N0 + Nmax, (-1)^Nq = parity, and
 *            sum 2m = two_m.  Species keys (Nq, 2M) ascending; blocks are the
 *            compatible (proton key, neutron key) pairs in that order; inside a
 *            key determinants ascend as unsigned integers (word n_words-1 most
 *            significant); row = block offset + ip * |neutron key| + in.
 *   two-body table (tbme): antisymmetrized V_{ab,cd}, a<b, c<d, one FP32 value
 *            per unordered {(ab),(cd)}.  Sectors by class (pp, pn, nn), then
 *            pair 2M, then pair parity; pairs lexicographic inside a sector and
 *            kept only if N_a + N_b <= N0(Z,N) - N0(Z-z, N-n) + Nmax; entries are
 *            the upper triangle, row-major.  ci_tbme_keys lists the keys.
 *   CSR      upper triangle including the diagonal; (i, j) is stored iff
 *            j >= i and the states differ in at most two nucleons, even when
 *            the value is zero; columns ascend inside a row.  row_ptr int64,
 *            col int32 (row index inside the basis), val FP32.  Diagonal and
 *            one-nucleon-difference sums are accumulated in FP64.
 *
 * Batches: n_probs > 1 builds independent bases side by side.  Basis b owns
 *   row_ptr[R_b .. R_b + D_b] with R_b = sum_{c<b} (D_c + 1); its values are
 *   positions in the concatenated col/val arrays (so row_ptr[R_b] is the
 *   number of entries of the bases before b).  tbme / grad_tbme of basis b
 *   start at T_b = sum_{c<b} n_tbme_c.
 *
 * Memory: every array argument marked "device" is caller-owned device memory
 * (for example a torch tensor on the GPU).  The two-body path allocates no
 * device memory: the index tables of a basis live in an arena the caller
 * passes to ci_basis_build, its partner lists in memory the caller passes to
 * ci_basis_build_lists (sizes from a size query and from ci_basis_list_bytes),
 * and the handle keeps pointers to these two buffers until ci_basis_free; the
 * caller keeps them alive (and unused by anything else) until the last call
 * on the handle has run.  No other call keeps a pointer to a caller array
 * after it returns.  All launches go to the given stream (hipStream_t; NULL =
 * the null stream).  The calls that read a count back and so synchronize the
 * stream are ci_basis_list_bytes, ci_hamiltonian_count(_full), the
 * three-body counts, ci_lanczos, ci_hamiltonian_tune and ci_probe_ceilings.
 *
 * Errors: every call returns CI_OK (0) or a negative CI_E* code; the message
 * of the last failure on the calling thread is ci_last_error().  Validation
 * errors are reported before any device call.
 */
#ifndef CI_H
#define CI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CI_OK 0
#define CI_EINVAL (-1)       /* null pointer, bad problem, bad index          */
#define CI_EUNSUPPORTED (-2) /* n_sps > 256 (more than 4 words), D >= 2^31,   */
                             /* a two-body sector too large for the index     */
#define CI_ESPACE (-3)       /* work buffer too small; sizes are in the info  */
#define CI_EHIP (-4)         /* HIP runtime error (message in ci_last_error)  */

typedef void* ci_stream; /* hipStream_t */

/* One problem: Z protons, N neutrons, Nmax excitation quanta above the lowest
 * filling, total 2M (two_m + Z + N must be even), parity +1 / -1, hw in MeV.
 * kinetic = 0: the one-body term is the oscillator energy (N + 3/2) hw of each
 * occupied orbit (diagonal); kinetic = 1: the one-body term is the oscillator
 * kinetic energy T (the paper's kinetic term, Sec. 2): on the diagonal
 * (hw/2)(2n + l + 3/2) per occupied orbit, and (hw/2) sqrt((n+1)(n+l+3/2))
 * between radial quantum numbers n and n + 1 of the same (l, j, m)
 * (one-nucleon differences). */
typedef struct {
    int32_t Z, N, nmax, two_m, parity;
    int32_t kinetic;
    double hw_mev;
} ci_problem;

/* Sizes of one basis (filled by ci_basis_plan / ci_basis_build). */
typedef struct {
    int32_t shell_max, n_sps, n_words, n0; /* S, orbits per species, words, N0 */
    int32_t n_pkeys, n_nkeys, n_blocks, n_sectors;
    int64_t n_psd, n_nsd; /* proton / neutron determinants */
    int64_t dim;          /* D */
    int64_t n_tbme;       /* two-body table length */
    int64_t row_ptr_offset; /* R_b */
    int64_t tbme_offset;    /* T_b */
    int64_t index_bytes;    /* device bytes of this basis' index tables (-1 until the lists are counted) */
    int64_t arena_bytes;    /* bytes of the arena of the whole build (the same in every entry) */
    int64_t list_bytes;     /* bytes of the partner lists of the whole build (-1 until counted) */
} ci_basis_info;

typedef struct ci_basis ci_basis; /* opaque */

/* Launch shapes of the row passes (count, fill) and of the adjoint, kept in
 * the handle.  Every shape computes the same result; only the time differs.
 * The row passes take one row per wavefront: either a grid that covers every
 * row once (row_grab = 0), or a persistent grid (as many workgroups as the
 * device holds at once) whose wavefronts take row_grab consecutive rows at a
 * time from a work counter until none are left.  The adjoint gives each
 * workgroup a tile of rows of one block -- tn = min(adj_tile_n, |Kn|) neutron
 * determinants times tp = max(1, adj_rows / tn) proton determinants -- whose
 * contributions are summed in one shared-memory table before they reach the
 * int64 fixed-point accumulators; the adjoint from stored words (ci_hamiltonian_vjp_keys)
 * has its own tile fields, adjk_rows, adjk_tile_n and adjk_persistent, which
 * ci_hamiltonian_tune tunes when it is given room for the words. */
typedef struct {
    int32_t row_waves;      /* wavefronts per workgroup of count and fill: 4 or 8 */
    int32_t row_grab;       /* 0: one grid over all rows; 1..4096: persistent, rows per grab */
    int32_t adj_rows;       /* adjoint: target rows per tile, 1..4096 */
    int32_t adj_tile_n;     /* adjoint: neutron determinants per tile, 1..4096 */
    int32_t adj_persistent; /* adjoint: 0 one workgroup per tile, 1 persistent workgroups */
    int32_t adjk_rows;      /* adjoint from stored words: target rows per tile, 1..4096 */
    int32_t adjk_tile_n;    /* adjoint from stored words: neutron determinants per tile, 1..4096 */
    int32_t adjk_persistent; /* adjoint from stored words: 0 one workgroup per tile, 1 persistent */
    int32_t row_xcd;        /* grids of rows or tiles (not persistent): 0 launch order; 1 each of the 8 XCDs */
                            /* (workgroup g runs on XCD g mod 8) takes one contiguous eighth of the grid   */
    int32_t adj_wide;       /* walking adjoint: 0 8 wavefronts sharing a 4096-slot table (three workgroups */
                            /* per CU); 1 16 wavefronts sharing a 16384-slot table (one per CU)            */
    int32_t adj_flush;      /* both adjoints: 0 each tile writes its table as records, summed per bucket by */
                            /* a second kernel; 1 each tile adds its table to int64 accumulators (device   */
                            /* atomics), then one conversion to FP32                                        */
} ci_tuning;

/* Thread-local text of the last error. */
const char* ci_last_error(void);

/* Host only, no device call: validates the problems and fills info[n_probs]
 * (the sizes that ci_basis_build will produce).  Sec. 2 (basis indexing). */
int ci_basis_plan(const ci_problem* probs, int32_t n_probs, ci_basis_info* info);

/* Host only: the two-body keys (a, b, c, d) of one problem in table order,
 * abcd [n_tbme][4] int32 host memory with room for cap rows. */
int ci_tbme_keys(const ci_problem* prob, int32_t* abcd, int64_t cap);

/* Builds the basis indexing (Sec. 2) of n_probs problems in three calls, the
 * count-then-allocate pattern of Sec. 4.1 applied to the index itself:
 *
 * 1. ci_basis_build with arena = NULL (size query, host only, no device
 *    call): plans the problems and fills info[n_probs]; info[b].arena_bytes is
 *    the arena the build needs (n_tbme, tbme_offset, index_bytes and
 *    list_bytes are -1 until the build).  The plan is kept for the calling
 *    thread, so that the build that follows with the same problems does not
 *    plan again.
 * 2. ci_basis_build with an arena (device memory, caller owned, at least
 *    arena_bytes, any contents): writes the host-built tables (determinants,
 *    keys, blocks, two-body pair index) into it with one copy (Sec. 5.2) and
 *    starts the count of the one- and two-nucleon partner lists on `stream`;
 *    fills info and returns the handle in *out without waiting for the
 *    device.  CI_ESPACE (and the plan kept) if arena_bytes is too small.
 * 3. ci_basis_list_bytes (synchronizes the stream: it reads the list lengths
 *    back) gives the bytes of the partner lists; ci_basis_build_lists fills
 *    them into caller memory of at least that size (asynchronous).
 *
 * Every later call on the handle needs the lists (CI_EINVAL before).  Work on
 * another stream than the build's must first synchronize with it. */
int ci_basis_build(const ci_problem* probs, int32_t n_probs, ci_basis_info* info, void* arena,
                   size_t arena_bytes, ci_basis** out, ci_stream stream);
int ci_basis_list_bytes(ci_basis* b, size_t* bytes, ci_stream stream);
int ci_basis_build_lists(ci_basis* b, void* lists, size_t bytes, ci_stream stream);

/* Frees the handle's host memory (NULL is allowed); no device call.  The
 * arena and the list memory stay the caller's: they may be reused once the
 * work queued on the handle has run (stream order). */
void ci_basis_free(ci_basis* b);

/* Count pass (Sec. 4.1): row_ptr (device, int64, sum_b (D_b + 1)) receives
 * the CSR row offsets of every basis; nnz (host, int64[n_probs]) the number
 * of stored entries per basis.  Synchronizes the stream (nnz is read back). */
int ci_hamiltonian_count(const ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream);

/* Fill pass (Sec. 2, Sec. 4.1): writes col (device int32) and val (device
 * FP32) of every stored entry at the positions given by row_ptr (from
 * ci_hamiltonian_count).  tbme: device FP32, concatenated tables.  Asynchronous. */
int ci_hamiltonian_fill(const ci_basis* b, const float* tbme, const int64_t* row_ptr,
                        int32_t* col, float* val, ci_stream stream);

/* Adjoint of the fill with respect to the two-body table: for L = sum_e
 * grad_val[e] * val[e], writes grad_tbme = dL/dtbme (device FP32, overwritten).
 * The pair / phase structure is recomputed, not stored.  The sums are in
 * fixed point: each contribution g becomes the integer rint(g * 2^s), with s
 * per basis from max |grad_val| over its entries and the rows of an adjoint
 * tile (so that no sum can overflow), the integers are added exactly (in LDS,
 * then in int64), and each total is scaled back and rounded once to FP32.
 * Integer sums have no order, so the result is the same bit for bit on every
 * run and for every adj_flush, adj_persistent, adj_wide and row_xcd at one
 * tile shape (adj_rows, adj_tile_n); other tile shapes round the contributions
 * on another grid (spacing at most 2^-(29 - ceil(log2 rows)) of max |grad_val|
 * per basis, rows = max(adj_rows, adj_tile_n)) and agree to that rounding.
 * grad_val must be finite.  work: device scratch of at least ci_vjp_work_bytes(b) bytes (int64
 * accumulators, tile records).  Asynchronous. */
int ci_hamiltonian_vjp(const ci_basis* b, const int64_t* row_ptr, const float* grad_val,
                       float* grad_tbme, void* work, size_t work_bytes, ci_stream stream);

/* The fill and its adjoint with the structure stored instead of recomputed:
 * ci_hamiltonian_fill_keys writes what ci_hamiltonian_fill writes (the same
 * col and val bits) and also keys (device uint32, one word per stored entry,
 * same positions): for an entry that is one two-body term, its position in
 * the basis' table (low 30 bits; all ones when no table element exists) and
 * its sign (bit 30); for the diagonal and one-nucleon differences (several
 * terms, Sec. 2), bit 31 and a record of the moved nucleon.  The words are
 * opaque to the caller and valid for this handle and row_ptr only.
 * ci_hamiltonian_vjp_keys computes what ci_hamiltonian_vjp computes from
 * those words (row_ptr, grad_val, grad_tbme, work as there) without walking
 * the partner lists again.  CI_EINVAL for null pointers, CI_EUNSUPPORTED when
 * a basis' table has 2^30 - 1 or more elements.  Asynchronous. */
int ci_hamiltonian_fill_keys(const ci_basis* b, const float* tbme, const int64_t* row_ptr, int32_t* col,
                             float* val, uint32_t* keys, ci_stream stream);
int ci_hamiltonian_vjp_keys(const ci_basis* b, const int64_t* row_ptr, const uint32_t* keys,
                            const float* grad_val, float* grad_tbme, void* work, size_t work_bytes,
                            ci_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * adjoint as ci_hamiltonian_vjp (same arguments without the work buffer, the
 * same bits at the same launch shapes), with its scratch (int64 accumulators, tile records and
 * histograms) in a fixed device array of the library, 64 MiB per GPU
 * (ci_vjp_noalloc_scratch_bytes), held from the first call on a GPU until the
 * process ends.  Calls nothing that allocates.  The table of the handle must
 * fit the scratch as int64 accumulators (n_tbme * 8 bytes, with room to spare;
 * else CI_ESPACE before any launch); the tile records get the rest (a tile
 * that finds no room adds its sums to the accumulators).  Every call on one
 * GPU shares the array: calls that overlap on one GPU (other streams, other
 * threads) race and give wrong results; order them.  Asynchronous. */
int ci_hamiltonian_vjp_noalloc(const ci_basis* b, const int64_t* row_ptr, const float* grad_val, float* grad_tbme,
                               ci_stream stream);
size_t ci_vjp_noalloc_scratch_bytes(void);

/* The same two passes for the FULL symmetric matrix (both triangles, every
 * (i, j) with d(i, j) <= 2, columns ascending in a row), as the eigensolver
 * needs it; same layout and batch conventions as above. */
int ci_hamiltonian_count_full(const ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream);
int ci_hamiltonian_fill_full(const ci_basis* b, const float* tbme, const int64_t* row_ptr,
                             int32_t* col, float* val, ci_stream stream);

/* ---- Matrix with a three-body term (paper Sec. 2: elements combine kinetic,
 * two-body and three-body terms; Sec. 4.1: count, then calculate and store
 * half of the symmetric matrix).  Stored entries: every (i, j), j >= i, whose
 * states differ in at most three nucleons (structural zeros included),
 * columns ascending.  Values: the one- and two-body part of
 * ci_hamiltonian_fill (zero three nucleons apart) plus the three-body part of
 * H3 = sum_{a<b<c, d<e<f} V_{abc,def} a+_a a+_b a+_c a_f a_e a_d by the
 * Slater-Condon rules (spectator sums for 0, 1, 2 nucleons apart; the
 * fermion phase of the other moves: holes removed from the column state in
 * ascending order, particles added in descending order).  The paper's
 * three-body elements come from its decoupling (Sec. 3); the interaction here
 * is synthetic (ci_v3).  Same row_ptr layout and batch conventions as the
 * two-body passes.  CI_EINVAL for null pointers or an unknown kind;
 * CI_EUNSUPPORTED when a problem has more than 128 nucleons. */
#define CI_V3_NONE 0      /* no three-body term (the two-body values on the d <= 3 structure) */
#define CI_V3_SYNTHETIC 1 /* V_{abc,def} for ascending triples of combined orbits: the (x+1)-th  */
                          /* output of splitmix64 started at seed, x = min(kb, kk) << 27 |       */
                          /* max(kb, kk), k = (a*512 + b)*512 + c per triple, mapped to          */
                          /* scale * (2u - 1) with u = top 53 bits / 2^53 (symmetric in bra/ket) */
#define CI_V3_IDENTITY 2  /* scale when the two triples are equal, else 0                        */
typedef struct {
    int32_t kind;
    uint64_t seed;
    double scale; /* MeV */
} ci_v3;

/* Count pass of the d <= 3 structure: row_ptr (device int64, sum of (D_b + 1)),
 * nnz (host int64[n_probs]).  Synchronizes the stream.  The first three-body
 * call on a handle also builds, and the handle keeps until ci_basis_free, an
 * index per species of the determinants within two nucleons of each other in
 * every key (device memory; a few MB to tens of MB); calls on one handle
 * must be ordered. */
int ci_hamiltonian3_count(ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream);
/* Fill pass: col (device int32), val (device FP32, FP64 sums) at row_ptr's
 * positions; tbme as for ci_hamiltonian_fill; v3 (host).  Asynchronous once
 * the handle holds its index (else it first builds it, synchronizing). */
int ci_hamiltonian3_fill(ci_basis* b, const float* tbme, const ci_v3* v3, const int64_t* row_ptr, int32_t* col,
                         float* val, ci_stream stream);
/* The same two passes for the FULL symmetric matrix with the three-body term
 * (both triangles, every (i, j) with d(i, j) <= 3, columns ascending), as
 * ci_lanczos takes it; every element is computed directly. */
int ci_hamiltonian3_count_full(ci_basis* b, int64_t* row_ptr, int64_t* nnz, ci_stream stream);
int ci_hamiltonian3_fill_full(ci_basis* b, const float* tbme, const ci_v3* v3, const int64_t* row_ptr,
                              int32_t* col, float* val, ci_stream stream);

/* y = H x for problem `prob` of the handle, H in full CSR form (row_ptr, col,
 * val from ci_hamiltonian_count_full / _fill_full; the problem's own row
 * segment is used).  x, y: device FP64 [D]; FP64 sums in a fixed order per
 * row (reproducible).  Asynchronous.  The step that follows construction in a
 * CI run (repeated products with a vector, paper Sec. 1-2). */
int ci_hamiltonian_spmv(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col,
                        const float* val, const double* x, double* y, ci_stream stream);

/* Lowest eigenvalue and eigenvector of H (full CSR as above) for problem
 * `prob` by the Lanczos method with full reorthogonalization (every new
 * vector is projected out of all earlier ones twice).  x0: device FP64 [D]
 * start vector (any nonzero vector).  Stops when the lowest Ritz value moves
 * by at most tol * max(1, |E|) between iterations, or after max_iter (1..4096)
 * iterations.  Outputs: *eval (host), *iters (host), evec (device FP64 [D],
 * unit norm).  work: device scratch of ci_lanczos_work_bytes(D, max_iter)
 * bytes.  Synchronizes the stream (the tridiagonal problem is solved on the
 * host each iteration).  CI_EINVAL for a zero start vector or bad sizes,
 * CI_ESPACE for a short work buffer. */
int ci_lanczos(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col,
               const float* val, const double* x0, int32_t max_iter, double tol, double* eval,
               int32_t* iters, double* evec, void* work, size_t work_bytes, ci_stream stream);

/* The same product and eigensolver on the matrix as the construction stores
 * it: the upper triangle only (row_ptr, col, val from ci_hamiltonian_count /
 * ci_hamiltonian_fill; half of the symmetric matrix, paper Sec. 2), with
 * H = U + (U - diag U)^T.  Every stored off-diagonal entry (i, j) is read
 * once and serves both y_i (a gather of x_j) and y_j (an FP64 device atomic
 * adding U_ij x_i), so y is reproducible to rounding only, not bit for bit.
 * ci_hamiltonian_spmv_upper overwrites y (it zeroes it first, on the
 * stream).  Arguments, errors and work size as for ci_hamiltonian_spmv and
 * ci_lanczos. */
int ci_hamiltonian_spmv_upper(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col,
                              const float* val, const double* x, double* y, ci_stream stream);
int ci_lanczos_upper(const ci_basis* b, int32_t prob, const int64_t* row_ptr, const int32_t* col,
                     const float* val, const double* x0, int32_t max_iter, double tol, double* eval,
                     int32_t* iters, double* evec, void* work, size_t work_bytes, ci_stream stream);

/* Bytes of work for ci_lanczos: (max_iter + 1) vectors of D doubles plus small buffers. */
size_t ci_lanczos_work_bytes(int64_t dim, int32_t max_iter);

/* Bytes of work needed by ci_hamiltonian_vjp for this handle. */
size_t ci_vjp_work_bytes(const ci_basis* b);

/* Autotuner (batched construction): times every candidate launch shape of
 * the fill and of both adjoints on the caller's buffers (one warm-up and
 * `reps` timed runs each, with HIP events on `stream`), keeps the fastest in
 * the handle, and remembers it for handles later built from the same problem
 * list in this process.  keys (device uint32 [nnz], may be NULL): room for the
 * stored words; with it the fill writes them once and the shapes of the
 * adjoint from stored words are tuned as well, else they stay as they are.
 * col, val (keys) and grad_tbme end up holding the results of a normal fill /
 * vjp.  Synchronizes the stream; not for use inside graph capture.  CI_EINVAL
 * for null pointers or reps < 1, CI_ESPACE for a short work buffer. */
int ci_hamiltonian_tune(ci_basis* b, const float* tbme, const int64_t* row_ptr, int32_t* col, float* val,
                        uint32_t* keys, const float* grad_val, float* grad_tbme, void* work, size_t work_bytes,
                        int32_t reps, ci_stream stream);

/* Current launch shapes of the handle; set them by hand (CI_EINVAL when a
 * field is out of range).  Calls on one handle share its work counter, so
 * they must be ordered (one stream, or synchronized between streams). */
int ci_basis_get_tuning(const ci_basis* b, ci_tuning* t);
int ci_basis_set_tuning(ci_basis* b, const ci_tuning* t);

/* ---- Three-body basis transformation (paper Sec. 3, the paper's own GPU
 * kernel): m-scheme elements of a three-body interaction, decoupled on request
 * from its coupled-JT form.
 *
 * Coupled basis: ordered triples (a, b, c) of oscillator orbitals (n, l, j) of
 * shells 0..n1max with N_a + N_b + N_c <= n3max, coupled as ((j_a j_b) J_ab,
 * j_c) J and ((1/2 1/2) T_ab, 1/2) T.  The input ("coupled", device FP32,
 * n_coupled values) holds one dense block per (bra triple, ket triple, J, T)
 * of equal parity, over channels (J_ab, T_ab) x (J_de, T_de); ci_threebody_keys
 * lists, per element in storage order, (t, t', 2J, 2T, 2J_ab, 2T_ab, 2J_de,
 * 2T_de).  A request is six int32 m-scheme orbits a b c d e f (orbit k of the
 * n_sps m-orbits of shells 0..n1max, ordered by N, l, 2j, 2m as for the basis;
 * proton k -> k, neutron k -> n_sps + k; isospin projection +1/2 for a
 * proton); its value is <abc|V|def> for the product states coupled in the
 * order (ab)c: the sum over J_ab, J_de, J, T_ab, T_de, T of the bra and ket
 * Clebsch-Gordan coefficients times the coupled element.  0 when M, M_T or
 * parity differ, when a triple lies beyond n3max, or for an index outside
 * [0, 2 n_sps). */
typedef struct ci_threebody ci_threebody; /* opaque: the layout and its device tables */

/* Host only: the sizes of the layout (same checks as ci_threebody_build). */
int ci_threebody_plan(int32_t n1max, int32_t n3max, int64_t* n_coupled, int32_t* n_triples);

/* Builds the layout and its device tables (one allocation, one copy).
 * CI_EINVAL unless 0 <= n1max <= 12 and 0 <= n3max <= 3 n1max;
 * CI_EUNSUPPORTED for more than 8192 triples. */
int ci_threebody_build(int32_t n1max, int32_t n3max, ci_threebody** out);
void ci_threebody_free(ci_threebody* t);
int ci_threebody_info(const ci_threebody* t, int64_t* n_coupled, int32_t* n_sps, int32_t* n_nlj,
                      int32_t* n_triples);
/* Host: keys [n_coupled][8] int32 (room for cap rows, else CI_ESPACE). */
int ci_threebody_keys(const ci_threebody* t, int32_t* keys, int64_t cap);
/* Host: nlj [n_nlj][3] = (N, l, 2j); morb [n_sps][2] = (orbital, 2m);
 * triples [n_triples][3] = orbitals (a, b, c). */
int ci_threebody_orbitals(const ci_threebody* t, int32_t* nlj, int32_t* morb, int32_t* triples);
/* out[r] (device FP32) = element of request r (device int32 [n][6]); one
 * request per lane (paper Sec. 3.2), FP64 sums.  work: null, or device memory
 * of ci_threebody_work_bytes(n) bytes (caller owned, no initial contents):
 * with it the requests are first grouped by an estimate of their cost and
 * the most expensive run first, so that the lanes of a wavefront run loops of
 * similar length; each result is the same either way (one lane sums one
 * request in a fixed order).  Asynchronous on stream; calls that share a work
 * buffer must be ordered.  CI_EINVAL for null pointers or n < 0, with work
 * for n > 2^31 - 1; CI_ESPACE for a short work buffer. */
size_t ci_threebody_work_bytes(int64_t n);
/* Host only: the Clebsch-Gordan coefficient <j1 m1 j2 m2 | J M> (all
 * arguments doubled, Condon-Shortley phases) by Racah's formula in long
 * double, the routine the decoupling's coefficient tables are built with; 0
 * outside the selection rules.  CI_EINVAL for a null out or a j outside
 * [0, 120]. */
int ci_clebsch_gordan(int32_t j1, int32_t m1, int32_t j2, int32_t m2, int32_t J, int32_t M, double* out);
int ci_threebody_decouple(const ci_threebody* t, const float* coupled, const int32_t* requests, int64_t n,
                          float* out, void* work, size_t work_bytes, ci_stream stream);

/* Machine ceilings measured on the current device (the roofline of the
 * construction kernels): streaming-store bandwidth over buf (device, caller
 * owned, at least 64 MiB; overwritten) in GB/s, and the rate of 64-bit
 * XOR + popcount difference-test steps (one step = XOR of two words, popcount,
 * add) per second, from 8 independent chains per lane.  Synchronizes the stream.
 * CI_ESPACE if bytes < 64 MiB. */
int ci_probe_ceilings(void* buf, size_t bytes, double* store_gbs, double* diff_steps_per_s,
                      ci_stream stream);

/* Number of problems in the handle; info of problem `prob`. */
int32_t ci_basis_count(const ci_basis* b);
int ci_basis_get_info(const ci_basis* b, int32_t prob, ci_basis_info* info);

/* Copies the basis states of problem `prob` to bits (device uint64
 * [D][2 * n_words], proton words then neutron words).  Asynchronous. */
int ci_basis_states(const ci_basis* b, int32_t prob, uint64_t* bits, ci_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* CI_H */
