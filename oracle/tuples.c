/* Orthogonal 8-tuple enumeration for the top-k form of the angle search.
 *
 * TEST INFRASTRUCTURE (CPU oracle).  Sec. 3.4 requires the chosen rows to form
 * an orthogonal set (T T^T diagonal).  Given, for each of the 8 DCT rows, a
 * ranked list of candidate integer vectors, this enumerates every choice of one
 * candidate per row whose 8 vectors are pairwise orthogonal, in lexicographic
 * order of list positions.  Plain depth-first search; the only speed-up is a
 * precomputed orthogonality bit matrix per pair of rows.
 *
 * Build: gcc -O2 -shared -fPIC tuples.c -o libtuples.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int nrows;
    const int *len;           /* len[r] */
    const int8_t *const *vec; /* vec[r][a*8 + e] */
    int words;                /* 64-bit words per bitset */
    uint64_t *ortho;          /* ortho[((r1*8 + r2)*kmax + a) * words + w] : bit b set if vec[r1][a] . vec[r2][b] == 0 */
    int kmax;
    int32_t *out;             /* out[count*8 + r] */
    int64_t cap;
    int64_t count;
} ctx_t;

static int dot8(const int8_t *u, const int8_t *v) {
    int s = 0;
    for (int e = 0; e < 8; ++e) s += (int)u[e] * (int)v[e];
    return s;
}

static uint64_t *bits(ctx_t *c, int r1, int r2, int a) {
    return c->ortho + ((size_t)(r1 * 8 + r2) * c->kmax + a) * c->words;
}

static void dfs(ctx_t *c, int row, int32_t *chosen, uint64_t *masks) {
    if (row == c->nrows) {
        if (c->count < c->cap) memcpy(c->out + c->count * 8, chosen, sizeof(int32_t) * 8);
        c->count++;
        return;
    }
    /* candidates for `row`: AND of the orthogonality rows of all chosen vectors */
    uint64_t *m = masks + (size_t)row * c->words;
    for (int w = 0; w < c->words; ++w) m[w] = ~(uint64_t)0;
    for (int r = 0; r < row; ++r) {
        const uint64_t *b = bits(c, r, row, chosen[r]);
        for (int w = 0; w < c->words; ++w) m[w] &= b[w];
    }
    for (int a = 0; a < c->len[row]; ++a) {
        if (!((m[a >> 6] >> (a & 63)) & 1)) continue;
        chosen[row] = a;
        dfs(c, row + 1, chosen, masks);
    }
}

/* lists: 8 pointers to (len[r] x 8) int8 arrays.  out: cap x 8 positions.
 * Returns the total number of tuples (may exceed cap; only cap are written),
 * or -1 on bad arguments / allocation failure. */
int64_t oracle_orthogonal_tuples(const int8_t *const *lists, const int *len,
                                 int32_t *out, int64_t cap) {
    if (!lists || !len || cap < 0 || (cap > 0 && !out)) return -1;
    int kmax = 0;
    for (int r = 0; r < 8; ++r) {
        if (len[r] < 0 || (len[r] > 0 && !lists[r])) return -1;
        if (len[r] > kmax) kmax = len[r];
    }
    if (kmax == 0) return 0;
    ctx_t c;
    c.nrows = 8; c.len = len; c.vec = lists; c.kmax = kmax;
    c.words = (kmax + 63) / 64;
    c.out = out; c.cap = cap; c.count = 0;
    c.ortho = (uint64_t *)calloc((size_t)64 * kmax * c.words, sizeof(uint64_t));
    uint64_t *masks = (uint64_t *)calloc((size_t)8 * c.words, sizeof(uint64_t));
    if (!c.ortho || !masks) { free(c.ortho); free(masks); return -1; }
    for (int r1 = 0; r1 < 8; ++r1)
        for (int r2 = r1 + 1; r2 < 8; ++r2)
            for (int a = 0; a < len[r1]; ++a) {
                uint64_t *b = bits(&c, r1, r2, a);
                for (int q = 0; q < len[r2]; ++q)
                    if (dot8(lists[r1] + 8 * a, lists[r2] + 8 * q) == 0)
                        b[q >> 6] |= (uint64_t)1 << (q & 63);
            }
    int32_t chosen[8] = {0};
    dfs(&c, 0, chosen, masks);
    free(c.ortho);
    free(masks);
    return c.count;
}
