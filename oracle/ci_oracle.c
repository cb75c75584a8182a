/*
 * ci_oracle.c -- plain FP64 CPU oracle for the M-scheme CI / No-Core Shell
 * Model Hamiltonian with a two-body interaction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, headers or tables with the HIP path.
 *
 * What it computes (paper, Sec. 2 "Overview of MFDn" and Sec. 4.1 "A Closer
 * Look at Matrix Construction"): the many-body basis is indexed, then every
 * nonzero element of the symmetric Hamiltonian is located and calculated as a
 * linear combination of kinetic(one-body) and two-body interaction terms, and
 * only half of the symmetric matrix is stored, in compressed-row form.
 *
 * The paper does not fix orbit order, bit layout, phases or the interaction
 * table layout; the readings used here (single-particle orbits, Nmax basis,
 * basis order, antisymmetrized two-body table, Slater-Condon rules) are the
 * textbook second-quantization definitions and are listed one by one in the
 * project's design notes.  Everything is done the slow, obvious way:
 *   - the basis is enumerated by a depth-first choice of occupied orbits;
 *   - row i is produced by testing EVERY column j >= i (O(D) per row);
 *   - every two-body element is found by binary search of the sorted key list.
 */
#include <stdint.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_MAXW 8 /* 64-bit words per species bitstring (n_sps <= 512) */

typedef struct {
    int N, n, l, j2, m2;
} orc_orbit;

typedef struct {
    int nq, m2;
} orc_key;

typedef struct {
    /* problem */
    int Z, NN, nmax, two_m, parity;
    int kinetic; /* 1: the one-body term is the oscillator kinetic energy T (diagonal and off-diagonal) */
    double hw;
    /* orbits */
    int S, nsps, W;
    orc_orbit* orb;
    double* spe; /* [2*nsps], combined index */
    int N0p, N0n, N0;
    /* species Slater determinants, grouped by key, colex inside a key */
    int npk, nnk;
    orc_key *pk, *nk;
    int64_t *pk_off, *nk_off; /* [npk+1], [nnk+1] */
    int64_t npsd, nnsd;
    uint64_t *psd, *nsd; /* [n][W] */
    /* blocks of compatible (proton key, neutron key) */
    int nblk;
    int *blk_kp, *blk_kn;
    int64_t* blk_off; /* [nblk+1] */
    int64_t D;
    uint64_t* st; /* [D][2W] : proton words then neutron words */
    /* two-body table */
    int64_t ntbme;
    int32_t* keys;     /* [ntbme][4] in table order */
    uint64_t* skey;    /* sorted packed keys */
    int64_t* sidx;     /* table index of each sorted key */
    double* V;         /* FP64 values in table order (may be NULL = all zero) */
    /* three-body interaction: kind 0 none, 1 synthetic, 2 identity */
    int v3_kind;
    uint64_t v3_seed;
    double v3_scale;
} orc_ctx;

/* ---------------------------------------------------------------- orbits */

/* Shell N of a harmonic-oscillator orbit holds (N+1)(N+2) states of one
 * species.  ntop(X): shell of the X-th nucleon when shells fill bottom-up;
 * n0(X): sum of the shells of the lowest X nucleons. */
static int shell_cap(int N) { return (N + 1) * (N + 2); }

static int ntop(int X)
{
    int N = 0, filled = 0;
    if (X <= 0) return 0;
    for (;;) {
        if (filled + shell_cap(N) >= X) return N;
        filled += shell_cap(N);
        N++;
    }
}

static int n0(int X)
{
    int s = 0, N = 0, left = X;
    while (left > 0) {
        int take = left < shell_cap(N) ? left : shell_cap(N);
        s += take * N;
        left -= take;
        N++;
    }
    return s;
}

/* orbits of shells 0..S in the order N, l, 2j, 2m (all ascending) */
static int make_orbits(int S, orc_orbit* out)
{
    int k = 0;
    for (int N = 0; N <= S; N++)
        for (int l = N % 2; l <= N; l += 2)
            for (int t = 0; t < 2; t++) {
                int j2 = (t == 0) ? 2 * l - 1 : 2 * l + 1;
                if (j2 < 0) continue;
                for (int m2 = -j2; m2 <= j2; m2 += 2) {
                    if (out) {
                        out[k].N = N;
                        out[k].n = (N - l) / 2;
                        out[k].l = l;
                        out[k].j2 = j2;
                        out[k].m2 = m2;
                    }
                    k++;
                }
            }
    return k;
}

/* ------------------------------------------------------- SD enumeration */

typedef struct {
    uint64_t* bits; /* growable [cap][W] */
    int* nq;
    int* m2;
    int64_t n, cap;
    int W;
} sdlist;

static void sd_push(sdlist* L, const uint64_t* w, int nq, int m2)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->bits = (uint64_t*)realloc(L->bits, (size_t)L->cap * L->W * sizeof(uint64_t));
        L->nq = (int*)realloc(L->nq, (size_t)L->cap * sizeof(int));
        L->m2 = (int*)realloc(L->m2, (size_t)L->cap * sizeof(int));
    }
    memcpy(L->bits + L->n * L->W, w, L->W * sizeof(uint64_t));
    L->nq[L->n] = nq;
    L->m2[L->n] = m2;
    L->n++;
}

/* choose `left` more orbits from index `start` on, keeping sum of N <= budget */
static void dfs(const orc_ctx* c, sdlist* L, uint64_t* w, int start, int left, int nq,
                int m2, int budget)
{
    if (left == 0) {
        sd_push(L, w, nq, m2);
        return;
    }
    for (int k = start; k < c->nsps; k++) {
        if (nq + c->orb[k].N > budget) continue;
        w[k / 64] |= (uint64_t)1 << (k % 64);
        dfs(c, L, w, k + 1, left - 1, nq + c->orb[k].N, m2 + c->orb[k].m2, budget);
        w[k / 64] &= ~((uint64_t)1 << (k % 64));
    }
}

static int key_cmp(const void* a, const void* b)
{
    const orc_key* x = (const orc_key*)a;
    const orc_key* y = (const orc_key*)b;
    if (x->nq != y->nq) return x->nq < y->nq ? -1 : 1;
    if (x->m2 != y->m2) return x->m2 < y->m2 ? -1 : 1;
    return 0;
}

/* colex order: the W-word string read as an unsigned integer, word W-1 most
 * significant */
static int g_W;
static int sd_cmp(const void* a, const void* b)
{
    const uint64_t* x = (const uint64_t*)a;
    const uint64_t* y = (const uint64_t*)b;
    for (int w = g_W - 1; w >= 0; w--)
        if (x[w] != y[w]) return x[w] < y[w] ? -1 : 1;
    return 0;
}

static int key_index(const orc_key* keys, int n, int nq, int m2)
{
    for (int k = 0; k < n; k++)
        if (keys[k].nq == nq && keys[k].m2 == m2) return k;
    return -1;
}

/* keep only keys that occur in some block; group SDs by key, colex inside */
static void species_table(const orc_ctx* c, const sdlist* L, const orc_key* keep, int nkeep,
                          int64_t** off_out, uint64_t** bits_out, int64_t* n_out)
{
    int W = c->W;
    int64_t* off = (int64_t*)calloc((size_t)nkeep + 1, sizeof(int64_t));
    int64_t* cnt = (int64_t*)calloc((size_t)nkeep, sizeof(int64_t));
    for (int64_t s = 0; s < L->n; s++) {
        int k = key_index(keep, nkeep, L->nq[s], L->m2[s]);
        if (k >= 0) cnt[k]++;
    }
    for (int k = 0; k < nkeep; k++) off[k + 1] = off[k] + cnt[k];
    uint64_t* bits = (uint64_t*)malloc((size_t)(off[nkeep] ? off[nkeep] : 1) * W * sizeof(uint64_t));
    memset(cnt, 0, (size_t)nkeep * sizeof(int64_t));
    for (int64_t s = 0; s < L->n; s++) {
        int k = key_index(keep, nkeep, L->nq[s], L->m2[s]);
        if (k < 0) continue;
        memcpy(bits + (off[k] + cnt[k]) * W, L->bits + s * W, W * sizeof(uint64_t));
        cnt[k]++;
    }
    g_W = W;
    for (int k = 0; k < nkeep; k++)
        qsort(bits + off[k] * W, (size_t)(off[k + 1] - off[k]), W * sizeof(uint64_t), sd_cmp);
    free(cnt);
    *off_out = off;
    *bits_out = bits;
    *n_out = off[nkeep];
}

/* distinct keys of an SD list, sorted */
static int distinct_keys(const sdlist* L, orc_key** out)
{
    orc_key* k = (orc_key*)malloc((size_t)(L->n ? L->n : 1) * sizeof(orc_key));
    int n = 0;
    for (int64_t s = 0; s < L->n; s++) {
        if (key_index(k, n, L->nq[s], L->m2[s]) < 0) {
            k[n].nq = L->nq[s];
            k[n].m2 = L->m2[s];
            n++;
        }
    }
    qsort(k, (size_t)n, sizeof(orc_key), key_cmp);
    *out = k;
    return n;
}

static int block_ok(const orc_ctx* c, orc_key p, orc_key q)
{
    int nq = p.nq + q.nq;
    if (nq > c->N0 + c->nmax) return 0;
    if (((nq % 2 == 0) ? 1 : -1) != c->parity) return 0;
    return p.m2 + q.m2 == c->two_m;
}

static void build_basis(orc_ctx* c)
{
    int W = c->W;
    uint64_t w[ORC_MAXW];
    sdlist Lp = {0}, Ln = {0};
    Lp.W = Ln.W = W;
    memset(w, 0, sizeof w);
    /* the most shells one species can hold: total budget minus the other
     * species at its lowest filling */
    dfs(c, &Lp, w, 0, c->Z, 0, 0, c->N0 + c->nmax - c->N0n);
    memset(w, 0, sizeof w);
    dfs(c, &Ln, w, 0, c->NN, 0, 0, c->N0 + c->nmax - c->N0p);

    orc_key *kp, *kn;
    int nkp = distinct_keys(&Lp, &kp), nkn = distinct_keys(&Ln, &kn);
    /* keys that take part in at least one block */
    int* usep = (int*)calloc((size_t)nkp + 1, sizeof(int));
    int* usen = (int*)calloc((size_t)nkn + 1, sizeof(int));
    for (int a = 0; a < nkp; a++)
        for (int b = 0; b < nkn; b++)
            if (block_ok(c, kp[a], kn[b])) usep[a] = usen[b] = 1;
    c->pk = (orc_key*)malloc((size_t)(nkp + 1) * sizeof(orc_key));
    c->nk = (orc_key*)malloc((size_t)(nkn + 1) * sizeof(orc_key));
    c->npk = c->nnk = 0;
    for (int a = 0; a < nkp; a++)
        if (usep[a]) c->pk[c->npk++] = kp[a];
    for (int b = 0; b < nkn; b++)
        if (usen[b]) c->nk[c->nnk++] = kn[b];
    free(usep);
    free(usen);
    free(kp);
    free(kn);

    species_table(c, &Lp, c->pk, c->npk, &c->pk_off, &c->psd, &c->npsd);
    species_table(c, &Ln, c->nk, c->nnk, &c->nk_off, &c->nsd, &c->nnsd);
    free(Lp.bits); free(Lp.nq); free(Lp.m2);
    free(Ln.bits); free(Ln.nq); free(Ln.m2);

    /* blocks in (proton key, neutron key) order; rows of a block run over the
     * proton SD (slow) then the neutron SD (fast) */
    c->blk_kp = (int*)malloc((size_t)(c->npk * c->nnk + 1) * sizeof(int));
    c->blk_kn = (int*)malloc((size_t)(c->npk * c->nnk + 1) * sizeof(int));
    c->blk_off = (int64_t*)malloc((size_t)(c->npk * c->nnk + 2) * sizeof(int64_t));
    c->nblk = 0;
    c->blk_off[0] = 0;
    for (int a = 0; a < c->npk; a++)
        for (int b = 0; b < c->nnk; b++)
            if (block_ok(c, c->pk[a], c->nk[b])) {
                int64_t sz = (c->pk_off[a + 1] - c->pk_off[a]) * (c->nk_off[b + 1] - c->nk_off[b]);
                c->blk_kp[c->nblk] = a;
                c->blk_kn[c->nblk] = b;
                c->blk_off[c->nblk + 1] = c->blk_off[c->nblk] + sz;
                c->nblk++;
            }
    c->D = c->blk_off[c->nblk];

    c->st = (uint64_t*)malloc((size_t)(c->D ? c->D : 1) * 2 * W * sizeof(uint64_t));
    int64_t i = 0;
    for (int bk = 0; bk < c->nblk; bk++) {
        int a = c->blk_kp[bk], b = c->blk_kn[bk];
        for (int64_t p = c->pk_off[a]; p < c->pk_off[a + 1]; p++)
            for (int64_t q = c->nk_off[b]; q < c->nk_off[b + 1]; q++) {
                memcpy(c->st + i * 2 * W, c->psd + p * W, W * sizeof(uint64_t));
                memcpy(c->st + i * 2 * W + W, c->nsd + q * W, W * sizeof(uint64_t));
                i++;
            }
    }
}

/* ------------------------------------------------------- two-body table */

/* combined index: proton orbit k -> k, neutron orbit k -> nsps + k */
static const orc_orbit* corb(const orc_ctx* c, int a) { return &c->orb[a % c->nsps]; }

static uint64_t pack4(int a, int b, int cc, int d)
{
    return ((uint64_t)a << 48) | ((uint64_t)b << 32) | ((uint64_t)cc << 16) | (uint64_t)d;
}

static const uint64_t* g_sort_keys;
static int idx_cmp(const void* x, const void* y)
{
    uint64_t a = g_sort_keys[*(const int64_t*)x], b = g_sort_keys[*(const int64_t*)y];
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Antisymmetrized, normalized matrix elements <ab|V|cd>, a<b, c<d, stored once
 * per unordered {bra, ket}.  Sectors: class (pp, pn, nn), then pair 2M, then
 * pair parity; pairs lexicographic inside a sector; upper triangle row-major.
 * A pair is kept only if N_a + N_b can occur in the basis:
 *     N_a + N_b <= N0(Z,N) - N0(Z - z, N - n) + Nmax   for z protons, n neutrons. */
static void build_tbme(orc_ctx* c)
{
    int n = c->nsps, n2 = 2 * n;
    int maxm = 0;
    for (int k = 0; k < n; k++)
        if (c->orb[k].m2 > maxm) maxm = c->orb[k].m2;
    int* pa = (int*)malloc((size_t)n2 * n2 * sizeof(int));
    int* pb = (int*)malloc((size_t)n2 * n2 * sizeof(int));
    /* first pass counts, second pass writes */
    for (int pass = 0; pass < 2; pass++) {
        int64_t t = 0;
        for (int cls = 0; cls < 3; cls++) {
            int z = (cls == 0) ? 2 : (cls == 1) ? 1 : 0;
            int nn = 2 - z;
            if (c->Z - z < 0 || c->NN - nn < 0) continue;
            int n2max = c->N0 - (n0(c->Z - z) + n0(c->NN - nn)) + c->nmax;
            for (int M = -2 * maxm; M <= 2 * maxm; M += 2)
                for (int par = 0; par < 2; par++) {
                    int np = 0;
                    for (int a = 0; a < n2; a++)
                        for (int b = a + 1; b < n2; b++) {
                            int ca = a < n ? 1 : 0, cb = b < n ? 1 : 0; /* 1 = proton */
                            if (ca + cb != z) continue;
                            const orc_orbit *oa = corb(c, a), *ob = corb(c, b);
                            if (oa->m2 + ob->m2 != M) continue;
                            if ((oa->N + ob->N) % 2 != par) continue;
                            if (oa->N + ob->N > n2max) continue;
                            pa[np] = a;
                            pb[np] = b;
                            np++;
                        }
                    for (int r = 0; r < np; r++)
                        for (int q = r; q < np; q++) {
                            if (pass == 1) {
                                c->keys[4 * t + 0] = pa[r];
                                c->keys[4 * t + 1] = pb[r];
                                c->keys[4 * t + 2] = pa[q];
                                c->keys[4 * t + 3] = pb[q];
                            }
                            t++;
                        }
                }
        }
        if (pass == 0) {
            c->ntbme = t;
            c->keys = (int32_t*)malloc((size_t)(t ? t : 1) * 4 * sizeof(int32_t));
        }
    }
    free(pa);
    free(pb);
    c->skey = (uint64_t*)malloc((size_t)(c->ntbme ? c->ntbme : 1) * sizeof(uint64_t));
    c->sidx = (int64_t*)malloc((size_t)(c->ntbme ? c->ntbme : 1) * sizeof(int64_t));
    uint64_t* raw = (uint64_t*)malloc((size_t)(c->ntbme ? c->ntbme : 1) * sizeof(uint64_t));
    for (int64_t t = 0; t < c->ntbme; t++) {
        raw[t] = pack4(c->keys[4 * t], c->keys[4 * t + 1], c->keys[4 * t + 2], c->keys[4 * t + 3]);
        c->sidx[t] = t;
    }
    g_sort_keys = raw;
    qsort(c->sidx, (size_t)c->ntbme, sizeof(int64_t), idx_cmp);
    for (int64_t t = 0; t < c->ntbme; t++) c->skey[t] = raw[c->sidx[t]];
    free(raw);
}

/* table index of canonical key (a<b, c<d, (a,b) <= (c,d)), or -1 */
static int64_t find_key(const orc_ctx* c, int a, int b, int cc, int d)
{
    uint64_t k = pack4(a, b, cc, d);
    int64_t lo = 0, hi = c->ntbme - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (c->skey[mid] == k) return c->sidx[mid];
        if (c->skey[mid] < k) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* Any ordering of (a,b,c,d) with a!=b, c!=d: each swap inside a pair flips the
 * sign (antisymmetry), bra and ket may be exchanged (real, Hermitian).
 * Returns the table index (or -1) and the sign. */
static int64_t lookup(const orc_ctx* c, int a, int b, int cc, int d, int* sign)
{
    int s = 1, t;
    if (a > b) { t = a; a = b; b = t; s = -s; }
    if (cc > d) { t = cc; cc = d; d = t; s = -s; }
    if (a > cc || (a == cc && b > d)) {
        t = a; a = cc; cc = t;
        t = b; b = d; d = t;
    }
    *sign = s;
    return find_key(c, a, b, cc, d);
}

static double Vget(const orc_ctx* c, int a, int b, int cc, int d)
{
    int s;
    int64_t k = lookup(c, a, b, cc, d, &s);
    if (k < 0 || !c->V) return 0.0;
    return s * c->V[k];
}

/* ------------------------------------------------------ matrix elements */

static int popc(uint64_t x) { return __builtin_popcountll(x); }

/* occupied combined indices of state i, ascending */
static int occupied(const orc_ctx* c, int64_t i, int* occ)
{
    int W = c->W, k = 0;
    const uint64_t* s = c->st + i * 2 * W;
    for (int sp = 0; sp < 2; sp++)
        for (int o = 0; o < c->nsps; o++)
            if ((s[sp * W + o / 64] >> (o % 64)) & 1) occ[k++] = sp * c->nsps + o;
    return k;
}

/* number of differing nucleons (half the popcount of the xor) */
static int ndiff(const orc_ctx* c, int64_t i, int64_t j)
{
    int W = c->W, x = 0;
    const uint64_t *a = c->st + i * 2 * W, *b = c->st + j * 2 * W;
    for (int w = 0; w < 2 * W; w++) x += popc(a[w] ^ b[w]);
    return x / 2;
}

static int in_list(const int* L, int n, int v)
{
    for (int k = 0; k < n; k++)
        if (L[k] == v) return 1;
    return 0;
}

static int count_below(const int* L, int n, int v)
{
    int k = 0;
    for (int t = 0; t < n; t++)
        if (L[t] < v) k++;
    return k;
}

/* Slater-Condon element <Phi_i | H | Phi_j> for d <= 2.  With gradient
 * output (g != NULL) it instead adds w * d<H_ij>/dV_k into g[k] for every
 * two-body term, and returns 0. */
/* Off-diagonal one-body element t_ab between combined orbits a != b of one
 * species: the oscillator kinetic energy T = -(hw/2) nabla^2 (lengths in
 * oscillator units) connects radial quantum numbers n and n + 1 of the same
 * (l, j, m), with <n+1 l|T|n l> = (hw/2) sqrt((n+1)(n+l+3/2)) (radial
 * functions positive near the origin); everything else is 0.  Its diagonal
 * (hw/2)(2n + l + 3/2) is in spe. */
static double onebody_offdiag(const orc_ctx* c, int a, int b)
{
    if (!c->kinetic || a == b || (a < c->nsps) != (b < c->nsps)) return 0.0;
    const orc_orbit *oa = corb(c, a), *ob = corb(c, b);
    if (oa->l != ob->l || oa->j2 != ob->j2 || oa->m2 != ob->m2) return 0.0;
    int lo = oa->n < ob->n ? oa->n : ob->n, hi = oa->n < ob->n ? ob->n : oa->n;
    if (hi != lo + 1) return 0.0;
    return 0.5 * c->hw * sqrt((double)(lo + 1) * (lo + oa->l + 1.5));
}

static double element(const orc_ctx* c, int64_t i, int64_t j, double* g, double w)
{
    int oi[2 * 64 * ORC_MAXW], oj[2 * 64 * ORC_MAXW];
    int ni = occupied(c, i, oi), nj = occupied(c, j, oj);
    int h[2] = {0, 0}, p[2] = {0, 0}, nh = 0, np = 0;
    for (int t = 0; t < nj; t++)
        if (!in_list(oi, ni, oj[t])) h[nh++] = oj[t]; /* holes: in j, not in i */
    for (int t = 0; t < ni; t++)
        if (!in_list(oj, nj, oi[t])) p[np++] = oi[t]; /* particles: in i, not in j */
    double v = 0.0;
    int s;
    int64_t k;
    if (nh == 0) {
        for (int a = 0; a < ni; a++) v += c->spe[oi[a]];
        for (int a = 0; a < ni; a++)
            for (int b = a + 1; b < ni; b++) {
                if (g) {
                    k = lookup(c, oi[a], oi[b], oi[a], oi[b], &s);
                    if (k >= 0) g[k] += s * w;
                } else {
                    v += Vget(c, oi[a], oi[b], oi[a], oi[b]);
                }
            }
        return g ? 0.0 : v;
    }
    if (nh == 1) {
        int lo = h[0] < p[0] ? h[0] : p[0], hi = h[0] < p[0] ? p[0] : h[0];
        int between = 0;
        for (int t = 0; t < nj; t++)
            if (oj[t] > lo && oj[t] < hi) between++;
        double sg = (between % 2) ? -1.0 : 1.0;
        for (int t = 0; t < nj; t++) {
            int kk = oj[t];
            if (kk == h[0]) continue;
            if (g) {
                k = lookup(c, p[0], kk, h[0], kk, &s);
                if (k >= 0) g[k] += sg * s * w;
            } else {
                v += Vget(c, p[0], kk, h[0], kk);
            }
        }
        if (!g) v += onebody_offdiag(c, p[0], h[0]);  /* a+_p a_h: the same phase */
        return g ? 0.0 : sg * v;
    }
    /* nh == 2: h[], p[] are ascending because the lists are */
    int T[2 * 64 * ORC_MAXW], nt = 0;
    for (int t = 0; t < nj; t++)
        if (oj[t] != h[0] && oj[t] != h[1]) T[nt++] = oj[t];
    int e = count_below(oj, nj, h[0]) + count_below(oj, nj, h[1]) - 1 + count_below(T, nt, p[0]) +
            count_below(T, nt, p[1]);
    double sg = (e % 2) ? -1.0 : 1.0;
    if (g) {
        k = lookup(c, p[0], p[1], h[0], h[1], &s);
        if (k >= 0) g[k] += sg * s * w;
        return 0.0;
    }
    return sg * Vget(c, p[0], p[1], h[0], h[1]);
}

/* ------------------------------------------------ three-body term (d <= 3)
 *
 * H3 = sum_{a<b<c, d<e<f} V_{abc,def} a+_a a+_b a+_c a_f a_e a_d with V
 * antisymmetric in each triple.  Between determinants that differ in d <= 3
 * nucleons (particles p in Phi_i, holes h in Phi_j, spectators T = the
 * orbits both hold) the Slater-Condon rules give
 *   d = 0: sum over occupied a<b<c of V_{abc,abc}
 *   d = 1: phase * sum over spectators k<l of V_{pkl,hkl}
 *   d = 2: phase * sum over spectators k of V_{p1 p2 k, h1 h2 k}
 *   d = 3: phase * V_{p1 p2 p3, h1 h2 h3}
 * with the same fermion phase as the one- and two-body moves: the holes
 * removed from Phi_j in ascending order, the particles added in descending
 * order.  The paper's three-body elements come from its decoupling (Sec. 3);
 * here the interaction is synthetic:
 *   kind 1: for ascending triples, the (x+1)-th output of the splitmix64
 *           generator (Steele, Lea & Flood 2014) started at `seed`, with
 *           x = min(kb, kk) << 27 | max(kb, kk), k = (a*512 + b)*512 + c for
 *           each triple, mapped to scale * (2u - 1), u = top 53 bits / 2^53
 *           (symmetric under bra <-> ket, so H stays symmetric);
 *   kind 2: scale when the two triples are equal, else 0 (then
 *           H3 = scale * A(A-1)(A-2)/6 on every A-nucleon state). */

static uint64_t splitmix64_at(uint64_t state, uint64_t k)
{
    uint64_t z = state + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double v3_sorted(const orc_ctx* c, int a, int b, int cc, int d, int e, int f)
{
    if (c->v3_kind == 2) return (a == d && b == e && cc == f) ? c->v3_scale : 0.0;
    uint64_t kb = ((uint64_t)a * 512 + (uint64_t)b) * 512 + (uint64_t)cc;
    uint64_t kk = ((uint64_t)d * 512 + (uint64_t)e) * 512 + (uint64_t)f;
    uint64_t lo = kb < kk ? kb : kk, hi = kb < kk ? kk : kb;
    uint64_t z = splitmix64_at(c->v3_seed, ((lo << 27) | hi) + 1);
    return c->v3_scale * (2.0 * ((double)(z >> 11) / 9007199254740992.0) - 1.0);
}

/* V_{abc,def} for triples in any order: each triple is sorted and every
 * transposition flips the sign; a repeated orbit gives 0. */
static double v3_any(const orc_ctx* c, int a, int b, int cc, int d, int e, int f)
{
    int x[3] = {a, b, cc}, y[3] = {d, e, f}, sg = 1;
    for (int r = 0; r < 2; r++)
        for (int q = 0; q < 2 - r; q++) {
            if (x[q] > x[q + 1]) { int t = x[q]; x[q] = x[q + 1]; x[q + 1] = t; sg = -sg; }
            if (y[q] > y[q + 1]) { int t = y[q]; y[q] = y[q + 1]; y[q + 1] = t; sg = -sg; }
        }
    if (x[0] == x[1] || x[1] == x[2] || y[0] == y[1] || y[1] == y[2]) return 0.0;
    return sg * v3_sorted(c, x[0], x[1], x[2], y[0], y[1], y[2]);
}

/* <Phi_i|H|Phi_j> with the three-body term, any i, j (0 beyond d = 3) */
static double element3(const orc_ctx* c, int64_t i, int64_t j)
{
    int oi[2 * 64 * ORC_MAXW], oj[2 * 64 * ORC_MAXW], T[2 * 64 * ORC_MAXW];
    int ni = occupied(c, i, oi), nj = occupied(c, j, oj);
    int h[3], p[3], nh = 0, np = 0, nt = 0;
    for (int t = 0; t < nj; t++)
        if (!in_list(oi, ni, oj[t])) {
            if (nh == 3) return 0.0;
            h[nh++] = oj[t];
        }
    for (int t = 0; t < ni; t++)
        if (!in_list(oj, nj, oi[t])) p[np++] = oi[t];
    double v = nh <= 2 ? element(c, i, j, NULL, 0.0) : 0.0;
    if (c->v3_kind == 0) return v;
    double w = 0.0;
    if (nh == 0) {
        for (int a = 0; a < ni; a++)
            for (int b = a + 1; b < ni; b++)
                for (int q = b + 1; q < ni; q++) w += v3_sorted(c, oi[a], oi[b], oi[q], oi[a], oi[b], oi[q]);
        return v + w;
    }
    for (int t = 0; t < nj; t++)
        if (!in_list(h, nh, oj[t])) T[nt++] = oj[t];
    int e = -nh * (nh - 1) / 2;
    for (int k = 0; k < nh; k++) e += count_below(oj, nj, h[k]) + count_below(T, nt, p[k]);
    double sg = (e % 2 != 0) ? -1.0 : 1.0;
    if (nh == 1) {
        for (int a = 0; a < nt; a++)
            for (int b = a + 1; b < nt; b++) w += v3_any(c, p[0], T[a], T[b], h[0], T[a], T[b]);
    } else if (nh == 2) {
        for (int a = 0; a < nt; a++) w += v3_any(c, p[0], p[1], T[a], h[0], h[1], T[a]);
    } else {
        w = v3_sorted(c, p[0], p[1], p[2], h[0], h[1], h[2]);
    }
    return v + sg * w;
}

/* ------------------------------------------------------------- public */

static void ctx_free(orc_ctx* c)
{
    if (!c) return;
    free(c->orb); free(c->spe);
    free(c->pk); free(c->nk); free(c->pk_off); free(c->nk_off);
    free(c->psd); free(c->nsd);
    free(c->blk_kp); free(c->blk_kn); free(c->blk_off);
    free(c->st);
    free(c->keys); free(c->skey); free(c->sidx); free(c->V);
    free(c);
}

/* Returns NULL for an invalid problem. */
void* orc_new(int Z, int N, int nmax, int two_m, int parity, double hw, int kinetic)
{
    if (Z < 0 || N < 0 || Z + N == 0 || nmax < 0 || (parity != 1 && parity != -1)) return NULL;
    if (kinetic != 0 && kinetic != 1) return NULL;
    if (((two_m + Z + N) % 2 + 2) % 2 != 0) return NULL;
    orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
    c->Z = Z; c->NN = N; c->nmax = nmax; c->two_m = two_m; c->parity = parity; c->hw = hw;
    c->kinetic = kinetic;
    int tz = ntop(Z), tn = ntop(N);
    c->S = (tz > tn ? tz : tn) + nmax;
    c->nsps = make_orbits(c->S, NULL);
    c->W = (c->nsps + 63) / 64;
    if (c->W > ORC_MAXW) { free(c); return NULL; }
    c->orb = (orc_orbit*)malloc((size_t)c->nsps * sizeof(orc_orbit));
    make_orbits(c->S, c->orb);
    c->spe = (double*)malloc((size_t)2 * c->nsps * sizeof(double));
    /* diagonal one-body energy: (N + 3/2) hw (oscillator energy), or with the
     * kinetic term <n l|T|n l> = (hw/2)(2n + l + 3/2) = (hw/2)(N + 3/2) */
    for (int a = 0; a < 2 * c->nsps; a++) c->spe[a] = (corb(c, a)->N + 1.5) * hw * (kinetic ? 0.5 : 1.0);
    c->N0p = n0(Z);
    c->N0n = n0(N);
    c->N0 = c->N0p + c->N0n;
    build_basis(c);
    build_tbme(c);
    return c;
}

void orc_free(void* h) { ctx_free((orc_ctx*)h); }

/* info[16]: S, nsps, W, N0, npk, nnk, nblk, npsd, nnsd, D, ntbme */
void orc_info(void* h, int64_t* info)
{
    orc_ctx* c = (orc_ctx*)h;
    info[0] = c->S; info[1] = c->nsps; info[2] = c->W; info[3] = c->N0;
    info[4] = c->npk; info[5] = c->nnk; info[6] = c->nblk;
    info[7] = c->npsd; info[8] = c->nnsd; info[9] = c->D; info[10] = c->ntbme;
}

/* orbit table [nsps][5]: N, n, l, 2j, 2m */
void orc_orbits(void* h, int32_t* out)
{
    orc_ctx* c = (orc_ctx*)h;
    for (int k = 0; k < c->nsps; k++) {
        out[5 * k] = c->orb[k].N; out[5 * k + 1] = c->orb[k].n; out[5 * k + 2] = c->orb[k].l;
        out[5 * k + 3] = c->orb[k].j2; out[5 * k + 4] = c->orb[k].m2;
    }
}

/* keys [npk][2], [nnk][2]; key offsets [npk+1], [nnk+1]; blocks [nblk][2]; block offsets [nblk+1] */
void orc_keys(void* h, int32_t* pk, int32_t* nk, int64_t* pk_off, int64_t* nk_off, int32_t* blk,
              int64_t* blk_off)
{
    orc_ctx* c = (orc_ctx*)h;
    for (int a = 0; a < c->npk; a++) { pk[2 * a] = c->pk[a].nq; pk[2 * a + 1] = c->pk[a].m2; }
    for (int b = 0; b < c->nnk; b++) { nk[2 * b] = c->nk[b].nq; nk[2 * b + 1] = c->nk[b].m2; }
    for (int a = 0; a <= c->npk; a++) pk_off[a] = c->pk_off[a];
    for (int b = 0; b <= c->nnk; b++) nk_off[b] = c->nk_off[b];
    for (int k = 0; k < c->nblk; k++) { blk[2 * k] = c->blk_kp[k]; blk[2 * k + 1] = c->blk_kn[k]; }
    for (int k = 0; k <= c->nblk; k++) blk_off[k] = c->blk_off[k];
}

/* species SD words [npsd][W], [nnsd][W] */
void orc_species(void* h, uint64_t* psd, uint64_t* nsd)
{
    orc_ctx* c = (orc_ctx*)h;
    memcpy(psd, c->psd, (size_t)c->npsd * c->W * sizeof(uint64_t));
    memcpy(nsd, c->nsd, (size_t)c->nnsd * c->W * sizeof(uint64_t));
}

/* basis states [D][2W] */
void orc_states(void* h, uint64_t* out)
{
    orc_ctx* c = (orc_ctx*)h;
    memcpy(out, c->st, (size_t)c->D * 2 * c->W * sizeof(uint64_t));
}

/* two-body keys [ntbme][4] in table order */
void orc_tbme_keys(void* h, int32_t* out)
{
    orc_ctx* c = (orc_ctx*)h;
    memcpy(out, c->keys, (size_t)c->ntbme * 4 * sizeof(int32_t));
}

/* FP64 two-body values in table order (copied); NULL clears to zero */
void orc_set_tbme(void* h, const double* v)
{
    orc_ctx* c = (orc_ctx*)h;
    free(c->V);
    c->V = NULL;
    if (!v) return;
    c->V = (double*)malloc((size_t)(c->ntbme ? c->ntbme : 1) * sizeof(double));
    memcpy(c->V, v, (size_t)c->ntbme * sizeof(double));
}

/* signed lookup of an arbitrary (a,b,c,d); 0 outside the stored table */
double orc_vget(void* h, int a, int b, int cc, int d) { return Vget((orc_ctx*)h, a, b, cc, d); }

/* number of stored entries in row i: columns j >= i with at most two
 * nucleons different (structural zeros included) */
static int64_t row_count(const orc_ctx* c, int64_t i)
{
    int64_t n = 0;
    for (int64_t j = i; j < c->D; j++)
        if (ndiff(c, i, j) <= 2) n++;
    return n;
}

/* counts[r] for each requested row */
void orc_row_counts(void* h, const int64_t* rows, int64_t nrows, int64_t* counts)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) counts[r] = row_count(c, rows[r]);
}

/* Entries of the requested rows, rows concatenated in the given order, columns
 * ascending inside a row.  `offs` are the caller's output offsets per row
 * (from orc_row_counts). */
void orc_rows(void* h, const int64_t* rows, int64_t nrows, const int64_t* offs, int32_t* cols,
              double* vals)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t i = rows[r], o = offs[r];
        for (int64_t j = i; j < c->D; j++) {
            if (ndiff(c, i, j) > 2) continue;
            cols[o] = (int32_t)j;
            if (vals) vals[o] = element(c, i, j, NULL, 0.0);
            o++;
        }
    }
}

/* The same for the full symmetric matrix: every column j (both triangles)
 * with at most two nucleons different, ascending; the elements below the
 * diagonal are computed directly (row i, column j < i), not copied. */
void orc_row_counts_full(void* h, const int64_t* rows, int64_t nrows, int64_t* counts)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t n = 0;
        for (int64_t j = 0; j < c->D; j++)
            if (ndiff(c, rows[r], j) <= 2) n++;
        counts[r] = n;
    }
}

void orc_rows_full(void* h, const int64_t* rows, int64_t nrows, const int64_t* offs, int32_t* cols,
                   double* vals)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t i = rows[r], o = offs[r];
        for (int64_t j = 0; j < c->D; j++) {
            if (ndiff(c, i, j) > 2) continue;
            cols[o] = (int32_t)j;
            if (vals) vals[o] = element(c, i, j, NULL, 0.0);
            o++;
        }
    }
}

/* Lower-triangle element <Phi_j|H|Phi_i> computed with the roles swapped:
 * used to check that the matrix is symmetric. */
double orc_element(void* h, int64_t i, int64_t j)
{
    orc_ctx* c = (orc_ctx*)h;
    if (ndiff(c, i, j) > 2) return 0.0;
    return element(c, i, j, NULL, 0.0);
}

/* Gradient of L = sum_e G_e * H_e over the stored entries of the given rows
 * with respect to the two-body table (FP64, table order, accumulated into g).
 * G holds the upstream values of those rows' entries in the orc_rows order. */
void orc_grad_rows(void* h, const int64_t* rows, int64_t nrows, const double* G, double* g)
{
    orc_ctx* c = (orc_ctx*)h;
    int64_t o = 0;
    for (int64_t r = 0; r < nrows; r++) {
        int64_t i = rows[r];
        for (int64_t j = i; j < c->D; j++) {
            if (ndiff(c, i, j) > 2) continue;
            element(c, i, j, g, G[o]);
            o++;
        }
    }
}

/* ------------------------------------------- three-body term: public */

void orc_set_v3(void* h, int kind, uint64_t seed, double scale)
{
    orc_ctx* c = (orc_ctx*)h;
    c->v3_kind = kind;
    c->v3_seed = seed;
    c->v3_scale = scale;
}

double orc_v3(void* h, int a, int b, int cc, int d, int e, int f)
{
    return v3_any((orc_ctx*)h, a, b, cc, d, e, f);
}

/* Stored entries with the three-body term: columns j >= i with at most three
 * nucleons different (structural zeros included), ascending. */
void orc_row_counts3(void* h, const int64_t* rows, int64_t nrows, int64_t* counts)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t n = 0;
        for (int64_t j = rows[r]; j < c->D; j++)
            if (ndiff(c, rows[r], j) <= 3) n++;
        counts[r] = n;
    }
}

void orc_rows3(void* h, const int64_t* rows, int64_t nrows, const int64_t* offs, int32_t* cols, double* vals)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t i = rows[r], o = offs[r];
        for (int64_t j = i; j < c->D; j++) {
            if (ndiff(c, i, j) > 3) continue;
            cols[o] = (int32_t)j;
            if (vals) vals[o] = element3(c, i, j);
            o++;
        }
    }
}

/* <Phi_i|H|Phi_j> with the three-body term for any i, j (both triangles) */
double orc_element3(void* h, int64_t i, int64_t j) { return element3((orc_ctx*)h, i, j); }

/* OpenMP threads of the row-parallel functions (the CPU-baseline timing runs
 * the oracle at all host threads and at one). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* The same for the full symmetric matrix with the three-body term: every
 * column j (both triangles) with at most three nucleons different. */
void orc_row_counts3_full(void* h, const int64_t* rows, int64_t nrows, int64_t* counts)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t n = 0;
        for (int64_t j = 0; j < c->D; j++)
            if (ndiff(c, rows[r], j) <= 3) n++;
        counts[r] = n;
    }
}

void orc_rows3_full(void* h, const int64_t* rows, int64_t nrows, const int64_t* offs, int32_t* cols, double* vals)
{
    orc_ctx* c = (orc_ctx*)h;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; r++) {
        int64_t i = rows[r], o = offs[r];
        for (int64_t j = 0; j < c->D; j++) {
            if (ndiff(c, i, j) > 3) continue;
            cols[o] = (int32_t)j;
            if (vals) vals[o] = element3(c, i, j);
            o++;
        }
    }
}
