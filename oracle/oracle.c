/*
 * CPU oracle for failure-less multi-pattern matching. TEST INFRASTRUCTURE ONLY: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load this file's
 * library. It shares no code with the HIP path.
 *
 * Both routines compute the match set of the problem statement (Section 2.2): for
 * patterns p_0..p_{N-1} and text T of length n, every pair (s, j) with
 * T[s .. s+|p_j|) == p_j, reported sorted by s, then j, as the 64-bit key (s << 32) | j.
 *
 *   orc_brute   -- the definition itself, bucketed by pattern length: for every start s
 *                  and every distinct length L, look T[s..s+L) up among the patterns of
 *                  length L (sorted, binary search) and report every id stored under it.
 *   orc_ac      -- textbook Aho-Corasick (the algorithm recalled in Section 2.2): goto
 *                  trie + failure links + dictionary (output) links, one left-to-right
 *                  pass, reporting every pattern that ends at each position. Threads
 *                  take chunks [a, b) and scan up to b + maxlen - 1 so that a match that
 *                  crosses the chunk end is still seen (the overlap rule of Section 2.2);
 *                  each chunk keeps only matches that start inside it.
 *
 * Bytes of the text that are >= the alphabet size have no goto transition anywhere,
 * so they simply never match (patterns are validated to lie inside the alphabet).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint64_t *v;
    uint64_t n, cap;
} vec64;

static int vpush(vec64 *a, uint64_t x) {
    if (a->n == a->cap) {
        uint64_t nc = a->cap ? a->cap * 2 : 1024;
        uint64_t *nv = (uint64_t *)realloc(a->v, nc * sizeof(uint64_t));
        if (!nv) return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = x;
    return 0;
}

static int cmp_u64(const void *x, const void *y) {
    uint64_t a = *(const uint64_t *)x, b = *(const uint64_t *)y;
    return (a > b) - (a < b);
}

/* Concatenate per-chunk key vectors (each already sorted, chunks in text order). */
static int gather(vec64 *parts, int nparts, uint64_t **out, uint64_t *count) {
    uint64_t tot = 0;
    for (int i = 0; i < nparts; i++) tot += parts[i].n;
    uint64_t *o = (uint64_t *)malloc((tot ? tot : 1) * sizeof(uint64_t));
    if (!o) return -1;
    uint64_t k = 0;
    for (int i = 0; i < nparts; i++) {
        if (parts[i].n) memcpy(o + k, parts[i].v, parts[i].n * sizeof(uint64_t));
        k += parts[i].n;
        free(parts[i].v);
    }
    free(parts);
    *out = o;
    *count = tot;
    return 0;
}

void orc_free(void *p) { free(p); }

int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------
 * Length-bucketed brute force.
 * ---------------------------------------------------------------------------------- */
static const uint8_t *g_bytes;
static const uint64_t *g_off;

static int cmp_pat(const void *x, const void *y) {
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    uint64_t la = g_off[a + 1] - g_off[a], lb = g_off[b + 1] - g_off[b];
    if (la != lb) return la < lb ? -1 : 1;
    int c = memcmp(g_bytes + g_off[a], g_bytes + g_off[b], la);
    if (c) return c;
    return (a > b) - (a < b);
}

int orc_brute(const uint8_t *pat_bytes, const uint64_t *pat_off, uint32_t n_pats,
              const uint8_t *text, uint64_t n, int nthreads,
              uint64_t **out, uint64_t *count) {
    uint32_t *ord = (uint32_t *)malloc((n_pats ? n_pats : 1) * sizeof(uint32_t));
    if (!ord) return -1;
    for (uint32_t i = 0; i < n_pats; i++) ord[i] = i;
    g_bytes = pat_bytes;
    g_off = pat_off;
    qsort(ord, n_pats, sizeof(uint32_t), cmp_pat);
    /* buckets: runs of equal length in ord */
    uint32_t nb = 0;
    uint32_t *bstart = (uint32_t *)malloc((n_pats + 1) * sizeof(uint32_t));
    uint64_t *blen = (uint64_t *)malloc((n_pats + 1) * sizeof(uint64_t));
    for (uint32_t i = 0; i < n_pats; i++) {
        uint64_t L = pat_off[ord[i] + 1] - pat_off[ord[i]];
        if (nb == 0 || blen[nb - 1] != L) {
            bstart[nb] = i;
            blen[nb] = L;
            nb++;
        }
    }
    bstart[nb] = n_pats;

    const uint64_t chunk = 1 << 16;
    int nparts = (int)((n + chunk - 1) / chunk);
    vec64 *parts = (vec64 *)calloc(nparts ? nparts : 1, sizeof(vec64));
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4) reduction(| : err)
#endif
    for (int c = 0; c < nparts; c++) {
        uint64_t a = (uint64_t)c * chunk, b = a + chunk < n ? a + chunk : n;
        vec64 *v = &parts[c];
        for (uint64_t s = a; s < b; s++) {
            uint64_t first = v->n;
            for (uint32_t k = 0; k < nb; k++) {
                uint64_t L = blen[k];
#ifdef ORC_MUTANT_BRUTE_END
                if (s + L >= n) break; /* planted mistake: drops a match ending at n-1 */
#else
                if (s + L > n) break; /* buckets ascend in length */
#endif
                /* lower bound of T[s..s+L) among ord[bstart[k] .. bstart[k+1]) */
                uint32_t lo = bstart[k], hi = bstart[k + 1];
                while (lo < hi) {
                    uint32_t mid = lo + (hi - lo) / 2;
                    if (memcmp(pat_bytes + pat_off[ord[mid]], text + s, L) < 0) lo = mid + 1;
                    else hi = mid;
                }
                for (uint32_t m = lo; m < bstart[k + 1]; m++) {
                    if (memcmp(pat_bytes + pat_off[ord[m]], text + s, L) != 0) break;
                    err |= vpush(v, (s << 32) | ord[m]);
                }
            }
            /* ids found at s come bucket by bucket; order them */
            if (v->n - first > 1) qsort(v->v + first, v->n - first, sizeof(uint64_t), cmp_u64);
        }
    }
    free(ord);
    free(bstart);
    free(blen);
    if (err) return -1;
    return gather(parts, nparts, out, count);
}

/* ------------------------------------------------------------------------------------
 * Textbook Aho-Corasick.
 * ---------------------------------------------------------------------------------- */
typedef struct {
    uint32_t n_nodes;
    uint32_t n_pats;
    uint32_t maxlen;
    /* goto function as an open-addressing hash: key = node * 256 + symbol + 1 */
    uint64_t *hkey;
    uint32_t *hval;
    uint64_t hmask;
    uint32_t *fail;      /* failure link */
    uint32_t *dict;      /* nearest proper suffix state that ends a pattern, or UINT32_MAX */
    uint32_t *out_head;  /* first pattern ending exactly here, or UINT32_MAX */
    uint32_t *out_next;  /* next pattern ending at the same state (per pattern id) */
    uint32_t *pat_len;
} ac_t;

static inline uint64_t hslot(uint64_t key, uint64_t mask) {
    key ^= key >> 29;
    key *= 0xbf58476d1ce4e5b9ULL;
    key ^= key >> 32;
    return key & mask;
}

static inline uint32_t ac_goto(const ac_t *A, uint32_t q, uint32_t c) {
    uint64_t key = (uint64_t)q * 256 + c + 1;
    uint64_t i = hslot(key, A->hmask);
    for (;;) {
        if (A->hkey[i] == key) return A->hval[i];
        if (A->hkey[i] == 0) return UINT32_MAX;
        i = (i + 1) & A->hmask;
    }
}

static void ac_set(ac_t *A, uint32_t q, uint32_t c, uint32_t child) {
    uint64_t key = (uint64_t)q * 256 + c + 1;
    uint64_t i = hslot(key, A->hmask);
    while (A->hkey[i] != 0) i = (i + 1) & A->hmask;
    A->hkey[i] = key;
    A->hval[i] = child;
}

void orc_ac_free(ac_t *A) {
    if (!A) return;
    free(A->hkey);
    free(A->hval);
    free(A->fail);
    free(A->dict);
    free(A->out_head);
    free(A->out_next);
    free(A->pat_len);
    free(A);
}

ac_t *orc_ac_build(const uint8_t *pat_bytes, const uint64_t *pat_off, uint32_t n_pats) {
    uint64_t total = 0;
    uint32_t maxlen = 0;
    for (uint32_t j = 0; j < n_pats; j++) {
        uint64_t L = pat_off[j + 1] - pat_off[j];
        total += L;
        if (L > maxlen) maxlen = (uint32_t)L;
    }
    ac_t *A = (ac_t *)calloc(1, sizeof(ac_t));
    uint64_t maxnodes = total + 1;
    uint64_t hcap = 16;
    while (hcap < 2 * maxnodes) hcap <<= 1;
    A->hmask = hcap - 1;
    A->hkey = (uint64_t *)calloc(hcap, sizeof(uint64_t));
    A->hval = (uint32_t *)malloc(hcap * sizeof(uint32_t));
    A->out_head = (uint32_t *)malloc(maxnodes * sizeof(uint32_t));
    A->out_next = (uint32_t *)malloc((n_pats ? n_pats : 1) * sizeof(uint32_t));
    A->pat_len = (uint32_t *)malloc((n_pats ? n_pats : 1) * sizeof(uint32_t));
    uint32_t *parent = (uint32_t *)malloc(maxnodes * sizeof(uint32_t));
    uint8_t *sym = (uint8_t *)malloc(maxnodes);
    if (!A->hkey || !A->hval || !A->out_head || !A->out_next || !parent || !sym) {
        free(parent);
        free(sym);
        orc_ac_free(A);
        return NULL;
    }
    for (uint64_t i = 0; i < maxnodes; i++) A->out_head[i] = UINT32_MAX;
    uint32_t nn = 1;
    parent[0] = 0;
    sym[0] = 0;
    /* insert patterns in reverse id order so each state's output list ascends by id */
    for (uint32_t jj = n_pats; jj-- > 0;) {
        uint32_t q = 0;
        uint64_t L = pat_off[jj + 1] - pat_off[jj];
        A->pat_len[jj] = (uint32_t)L;
        for (uint64_t d = 0; d < L; d++) {
            uint32_t c = pat_bytes[pat_off[jj] + d];
            uint32_t nx = ac_goto(A, q, c);
            if (nx == UINT32_MAX) {
                nx = nn++;
                parent[nx] = q;
                sym[nx] = (uint8_t)c;
                ac_set(A, q, c, nx);
            }
            q = nx;
        }
        A->out_next[jj] = A->out_head[q];
        A->out_head[q] = jj;
    }
    A->n_nodes = nn;
    A->n_pats = n_pats;
    A->maxlen = maxlen;
    /* nodes in breadth-first order: bucket by depth using parent links */
    uint32_t *depth = (uint32_t *)malloc(nn * sizeof(uint32_t));
    uint32_t *order = (uint32_t *)malloc(nn * sizeof(uint32_t));
    uint32_t *cnt = (uint32_t *)calloc(maxlen + 2, sizeof(uint32_t));
    depth[0] = 0;
    /* a child is always created after its parent, so one increasing pass suffices */
    for (uint32_t v = 1; v < nn; v++) depth[v] = depth[parent[v]] + 1;
    for (uint32_t v = 0; v < nn; v++) cnt[depth[v] + 1]++;
    for (uint32_t d = 1; d <= maxlen + 1; d++) cnt[d] += cnt[d - 1];
    for (uint32_t v = 0; v < nn; v++) order[cnt[depth[v]]++] = v;
    A->fail = (uint32_t *)malloc(nn * sizeof(uint32_t));
    A->dict = (uint32_t *)malloc(nn * sizeof(uint32_t));
    A->fail[0] = 0;
    A->dict[0] = UINT32_MAX;
    for (uint32_t i = 1; i < nn; i++) {
        uint32_t v = order[i];
        uint32_t p = parent[v], c = sym[v];
        uint32_t f;
        if (p == 0) {
            f = 0; /* first-level failure links point at the root */
#ifdef ORC_MUTANT_ROOT_FAIL
        } else if (1) {
            f = 0; /* planted mistake: every failure link to the root */
#endif
        } else {
            /* longest proper suffix of v's string that is a trie state */
            uint32_t r = A->fail[p];
            for (;;) {
                uint32_t g = ac_goto(A, r, c);
                if (g != UINT32_MAX) { f = g; break; }
                if (r == 0) { f = 0; break; }
                r = A->fail[r];
            }
        }
        A->fail[v] = f;
        A->dict[v] = (A->out_head[f] != UINT32_MAX) ? f : A->dict[f];
    }
    free(depth);
    free(order);
    free(cnt);
    free(parent);
    free(sym);
    return A;
}

uint32_t orc_ac_nodes(const ac_t *A) { return A->n_nodes; }

static int ac_emit(const ac_t *A, uint32_t t, uint64_t e, uint64_t a, uint64_t b, vec64 *v) {
    int err = 0;
    for (uint32_t j = A->out_head[t]; j != UINT32_MAX; j = A->out_next[j]) {
        uint64_t s = e + 1 - A->pat_len[j];
        if (s >= a && s < b) err |= vpush(v, (s << 32) | j);
    }
    return err;
}

int orc_ac_scan(const ac_t *A, const uint8_t *text, uint64_t n, uint32_t alphabet,
                uint64_t chunk, int nthreads, uint64_t **out, uint64_t *count) {
    if (chunk == 0) chunk = 1 << 22;
    int nparts = (int)((n + chunk - 1) / chunk);
    vec64 *parts = (vec64 *)calloc(nparts ? nparts : 1, sizeof(vec64));
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
#endif
    for (int c = 0; c < nparts; c++) {
        uint64_t a = (uint64_t)c * chunk, b = a + chunk < n ? a + chunk : n;
#ifdef ORC_MUTANT_SHORT_OVERLAP
        uint64_t e_end = b + (A->maxlen > 1 ? A->maxlen - 2 : 0); /* planted mistake */
#else
        uint64_t e_end = b + (A->maxlen ? A->maxlen - 1 : 0);
#endif
        if (e_end > n) e_end = n;
        vec64 *v = &parts[c];
        uint32_t q = 0;
        for (uint64_t e = a; e < e_end; e++) {
            uint32_t ch = text[e];
            if (ch >= alphabet) {
                q = 0; /* no state has a transition on this byte */
                continue;
            }
            for (;;) {
                uint32_t g = ac_goto(A, q, ch);
                if (g != UINT32_MAX) { q = g; break; }
                if (q == 0) break;
                q = A->fail[q];
            }
            /* report every pattern ending at e: the state itself, then dictionary links */
            uint32_t t = (A->out_head[q] != UINT32_MAX) ? q : A->dict[q];
            while (t != UINT32_MAX) {
                err |= ac_emit(A, t, e, a, b, v);
#ifdef ORC_MUTANT_NO_DICT
                break; /* planted mistake: only the longest pattern ending at e */
#endif
                t = A->dict[t];
            }
        }
        if (v->n > 1) qsort(v->v, v->n, sizeof(uint64_t), cmp_u64);
    }
    if (err) return -1;
    return gather(parts, nparts, out, count);
}
