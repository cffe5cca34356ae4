/*
 * slm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately simple CPU implementation of the
 * Synchronised Louvain Method (Chiem, Havelange & Van Dooren, "A parallel
 * implementation of the Synchronised Louvain Method", arXiv 1702.04645),
 * written from the paper: Algorithm 1 (the level loop), Sec. 3.1 ASSIGN,
 * Sec. 3.2 COMPONENTS, Sec. 3.3 POSITIVE, Sec. 3.4 MAXIMAL, Sec. 3.5
 * AGGREGATE, the appendix pseudocode of the three steps, and the weighted
 * modularity Q_w of Sec. 2.4.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The GPU library shares no code with it.
 *
 * Conventions (the paper leaves them open; each is a stated reading):
 *  - The graph is undirected: a symmetric CSR matrix A with positive integer
 *    weights, columns strictly ascending in each row, the diagonal A_ii stored
 *    once.  k_i = sum_j A_ij (row sum, diagonal included), M2 = sum_i k_i.
 *    For a symmetric W the weighted modularity of Sec. 2.4 has m_w = M2.
 *  - Every gain is an exact int64 integer, a positive multiple of the
 *    modularity change (M2^2/2 times it), so argmax and sign tests are exact:
 *      pair(i,j)  = M2*A_ij - k_i*k_j                     (ASSIGN, re-pointing)
 *      join(i,C)  = M2*w(i,C) - k_i*S_C                   (i not in C)
 *      stay(i)    = M2*w(i,c_i\i) - k_i*(S_ci - k_i)      (local gain g(i))
 *      move(B:c->D) = M2*(w(B,D) - w(B,c\B)) - S_B*(S_D - S_c + S_B)
 *      split(P1,P2) = S_P1*S_P2 - M2*w(P1,P2)
 *    with S_X = sum of k over X and w(X,Y) = sum of A_uv, u in X, v in Y.
 *  - Ties: lowest node id for node choices, lowest canonical label for
 *    community choices, lowest (first, second) cut node for splits.
 *  - Canonical labels number the communities 0..n_c-1 in increasing order of
 *    their smallest member.
 *  - Strict tests: ASSIGN needs pair > 0, MAXIMAL needs join > stay, a tail
 *    move needs move > 0, a community is split while some g(i) < 0.
 *  - The acceptance draw of MAXIMAL is u32(seed, level, round, node): the high
 *    32 bits of one SplitMix64 output (Steele, Lea & Flood 2014), accepted iff
 *    u32 < accept_p (accept_p is a Q32 threshold; 2^31 is p = 1/2).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

typedef struct {
    int64_t n;
    const int64_t *rp;
    const int32_t *col;
    const int32_t *w;
} graph;

/* The null model of the quality function (Sec. 2.2 energy with alpha and
 * beta, Sec. 2.3 null models, Sec. 2.4 weighted modularity with out- and
 * in-strengths).  Every gain is
 *     A * w(P,R) - nu(P,R),   nu(P,R) = X_P * X_R - Y_P * Y_R
 * for merging disjoint node sets P and R, where w(P,R) sums the symmetric
 * matrix the level runs on, X and Y sum the per-node strengths x and y, and
 * A > 0 scales the edge term.  The undirected modularity of the rest of this
 * file is x = k, y = 0, A = M2.  y == NULL means y = 0. */
typedef struct {
    const int64_t *x;
    const int64_t *y;
    int64_t A;
} nullm;

static inline int64_t ny(const nullm *nm, int64_t i)
{
    return nm->y ? nm->y[i] : 0;
}

static void *xmalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

static void *xcalloc(size_t count, size_t size)
{
    void *p = calloc(count ? count : 1, size ? size : 1);
    if (!p) abort();
    return p;
}

/* ------------------------------------------------------------------------ */
/* Counter-based draw (Sec. 3.4: each maximal correction is accepted with a */
/* probability p; the generator itself is not given, so SplitMix64 is used). */
/* ------------------------------------------------------------------------ */

/* SplitMix64 output function applied to a state value. */
uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The (ctr+1)-th SplitMix64 output of the stream seeded with `seed`, where
 * ctr packs (level:16 | round:16 | node:32); the high half is returned. */
uint32_t or_draw(uint64_t seed, int32_t level, int32_t round, int32_t node)
{
    uint64_t ctr = ((uint64_t)(uint16_t)level << 48) |
                   ((uint64_t)(uint16_t)round << 32) | (uint64_t)(uint32_t)node;
    uint64_t state = seed + (ctr + 1ULL) * 0x9E3779B97F4A7C15ULL;
    return (uint32_t)(or_mix64(state) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Strengths (Sec. 2.4: s_i, m_w)                                             */
/* ------------------------------------------------------------------------ */

int64_t or_strength(int64_t n, const int64_t *rp, const int32_t *col,
                    const int32_t *w, int64_t *k_out)
{
    (void)col;
    int64_t m2 = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t s = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) s += w[e];
        k_out[i] = s;
        m2 += s;
    }
    return m2;
}

/* ------------------------------------------------------------------------ */
/* ASSIGN (Sec. 3.1 and the appendix ASSIGN): best neighbour of every node.  */
/* ------------------------------------------------------------------------ */

void or_assign_nm(int64_t n, const int64_t *rp, const int32_t *col,
                  const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                  int32_t *a_out)
{
    const nullm nm = {x, y, A};
    for (int64_t i = 0; i < n; i++) {
        int64_t best_j = -1, best_key = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int64_t j = col[e];
            if (j == i) continue;
            /* pair(i,j): the gain of merging the singletons {i} and {j} */
            int64_t key = A * (int64_t)w[e] - (x[i] * x[j] - ny(&nm, i) * ny(&nm, j));
            if (best_j < 0 || key > best_key || (key == best_key && j < best_j)) {
                best_j = j;
                best_key = key;
            }
        }
        /* a node whose best gain is not positive is self-assigned */
        a_out[i] = (best_j >= 0 && best_key > 0) ? (int32_t)best_j : (int32_t)i;
    }
}

void or_assign(int64_t n, const int64_t *rp, const int32_t *col,
               const int32_t *w, const int64_t *k, int64_t m2, int32_t *a_out)
{
    or_assign_nm(n, rp, col, w, k, NULL, m2, a_out);
}

/* ------------------------------------------------------------------------ */
/* COMPONENTS (Sec. 3.2): weakly connected components of T = {(i, a(i))}.   */
/* ------------------------------------------------------------------------ */

static int64_t uf_find(int64_t *parent, int64_t x)
{
    int64_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) {
        int64_t nx = parent[x];
        parent[x] = r;
        x = nx;
    }
    return r;
}

/* Canonical labels (communities numbered by smallest member) and the cycle
 * flag of every node; returns the number of communities. */
int64_t or_components(int64_t n, const int32_t *a, int32_t *lab_out,
                      uint8_t *on_cycle_out)
{
    int64_t *parent = xmalloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) parent[i] = i;
    for (int64_t i = 0; i < n; i++) {
        int64_t r1 = uf_find(parent, i), r2 = uf_find(parent, a[i]);
        if (r1 != r2) parent[r1 < r2 ? r2 : r1] = r1 < r2 ? r1 : r2;
    }
    /* scanning ids upwards meets every component first at its smallest member */
    int32_t *root_label = xmalloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) root_label[i] = -1;
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) {
        int64_t r = uf_find(parent, i);
        if (root_label[r] < 0) root_label[r] = (int32_t)nc++;
        lab_out[i] = root_label[r];
    }
    if (on_cycle_out) {
        /* walk from every unvisited node; a walk that meets its own trail
         * has found a cycle (state 1 = on the current trail, 2 = finished) */
        uint8_t *state = xcalloc((size_t)n, 1);
        memset(on_cycle_out, 0, (size_t)n);
        for (int64_t s = 0; s < n; s++) {
            if (state[s]) continue;
            int64_t x = s;
            while (state[x] == 0) {
                state[x] = 1;
                x = a[x];
            }
            if (state[x] == 1) {
                int64_t y = x;
                do {
                    on_cycle_out[y] = 1;
                    y = a[y];
                } while (y != x);
            }
            x = s;
            while (state[x] == 1) {
                state[x] = 2;
                x = a[x];
            }
        }
        free(state);
    }
    free(root_label);
    free(parent);
    return nc;
}

/* ------------------------------------------------------------------------ */
/* Community totals and local gains (Sec. 3.3, appendix POSITIVE).           */
/* ------------------------------------------------------------------------ */

/* S_C for every community C of the labelling `lab` (the sum of k, or of any
 * per-node strength, over its members). */
static void community_totals(int64_t n, const int64_t *k, const int32_t *lab,
                             int64_t nc, int64_t *sig)
{
    for (int64_t c = 0; c < nc; c++) sig[c] = 0;
    for (int64_t i = 0; i < n; i++) sig[lab[i]] += k[i];
}

/* X_C and Y_C of every community (Y all zero when the model has no y). */
static void null_totals(int64_t n, const nullm *nm, const int32_t *lab, int64_t nc,
                        int64_t *sx, int64_t *sy)
{
    community_totals(n, nm->x, lab, nc, sx);
    if (nm->y) community_totals(n, nm->y, lab, nc, sy);
    else for (int64_t c = 0; c < nc; c++) sy[c] = 0;
}

/* g(i) = stay(i): the gain of i being in its community rather than alone. */
void or_local_gain_nm(int64_t n, const int64_t *rp, const int32_t *col,
                      const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                      const int32_t *lab, int64_t nc, int64_t *g_out)
{
    const nullm nm = {x, y, A};
    int64_t *sx = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    int64_t *sy = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    null_totals(n, &nm, lab, nc, sx, sy);
    for (int64_t i = 0; i < n; i++) {
        int64_t w_in = 0; /* w(i, c_i \ i) */
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
            if (col[e] != i && lab[col[e]] == lab[i]) w_in += w[e];
        int32_t c = lab[i];
        g_out[i] = A * w_in - (x[i] * (sx[c] - x[i]) - ny(&nm, i) * (sy[c] - ny(&nm, i)));
    }
    free(sy);
    free(sx);
}

void or_local_gain(int64_t n, const int64_t *rp, const int32_t *col,
                   const int32_t *w, const int64_t *k, int64_t m2,
                   const int32_t *lab, int64_t nc, int64_t *g_out)
{
    or_local_gain_nm(n, rp, col, w, k, NULL, m2, lab, nc, g_out);
}

/* ------------------------------------------------------------------------ */
/* POSITIVE (Sec. 3.3): split every community holding a node of negative   */
/* local gain by its best bisection of the assignment graph, until no node  */
/* has a negative local gain.                                               */
/* ------------------------------------------------------------------------ */

/* Work space shared by the split search of one part. */
typedef struct {
    int64_t n;
    int32_t *part;     /* part id of every node                          */
    uint8_t *cyc;      /* on the cycle of its part                       */
    int32_t *tin;      /* DFS entry time inside the part                 */
    int32_t *tout;     /* DFS exit time (one past the last descendant)   */
    int32_t *order;    /* order[t] = node entered at time t              */
    int32_t *pos;      /* cycle position of the hanging tree of a node   */
    int32_t *head;     /* children lists: head[u], next[v]               */
    int32_t *next;
    int64_t *sub;      /* sum of x over the subtree                      */
    int64_t *suby;     /* sum of y over the subtree                      */
    int64_t *gl;       /* local gain                                     */
} pwork;

/* Members of the part holding node `s`, following pointers both ways is not
 * needed: the caller passes the member list. Builds cycle order, DFS times
 * and subtree sums for the members `mem[0..m-1]` of one part. Returns the
 * cycle length; the cycle in pointer order is written to `cycle`. */
static int64_t part_structure(const int32_t *a, const nullm *nm, pwork *W,
                              const int32_t *mem, int64_t m, int32_t *cycle)
{
    /* cycle: follow pointers from any member for m steps; the node reached
     * lies on the cycle; then walk the cycle once */
    int64_t x = mem[0];
    for (int64_t s = 0; s < m; s++) x = a[x];
    int64_t L = 0;
    int64_t y = x;
    do {
        L++;
        y = a[y];
    } while (y != x);
    for (int64_t s = 0; s < m; s++) W->cyc[mem[s]] = 0;
    /* start the cycle at its smallest node */
    int64_t start = x;
    y = x;
    for (int64_t s = 0; s < L; s++) {
        if (y < start) start = y;
        y = a[y];
    }
    y = start;
    for (int64_t s = 0; s < L; s++) {
        cycle[s] = (int32_t)y;
        W->cyc[y] = 1;
        W->pos[y] = (int32_t)s;
        y = a[y];
    }
    /* children lists of the hanging trees, in increasing id order */
    for (int64_t s = 0; s < m; s++) W->head[mem[s]] = -1;
    for (int64_t s = m - 1; s >= 0; s--) {
        int32_t u = mem[s];
        if (W->cyc[u]) continue;
        W->next[u] = W->head[a[u]];
        W->head[a[u]] = u;
    }
    /* iterative DFS from every cycle node in cycle order */
    int32_t *stack = xmalloc((size_t)m * sizeof(int32_t));
    int64_t t = 0;
    for (int64_t s = 0; s < L; s++) {
        int64_t sp = 0;
        stack[sp++] = cycle[s];
        W->tin[cycle[s]] = (int32_t)t;
        W->order[t++] = cycle[s];
        W->pos[cycle[s]] = (int32_t)s;
        /* head[] doubles as the per-node child cursor during the DFS */
        while (sp > 0) {
            int32_t u = stack[sp - 1];
            int32_t c = W->head[u];
            if (c >= 0) {
                W->head[u] = W->next[c];
                W->tin[c] = (int32_t)t;
                W->order[t++] = c;
                W->pos[c] = (int32_t)s;
                stack[sp++] = c;
            } else {
                W->tout[u] = (int32_t)t;
                sp--;
            }
        }
    }
    free(stack);
    /* subtree sums in reverse DFS order (children are entered after parents) */
    for (int64_t s = 0; s < m; s++) {
        W->sub[mem[s]] = nm->x[mem[s]];
        W->suby[mem[s]] = ny(nm, mem[s]);
    }
    for (int64_t s = t - 1; s >= 0; s--) {
        int32_t u = W->order[s];
        if (!W->cyc[u]) {
            W->sub[a[u]] += W->sub[u];
            W->suby[a[u]] += W->suby[u];
        }
    }
    return L;
}

/* Local gains of the members of one part, from the part's own totals. */
static void part_gains(const graph *g, const nullm *nm, pwork *W,
                       const int32_t *mem, int64_t m)
{
    int32_t p = W->part[mem[0]];
    int64_t sp = 0, spy = 0;
    for (int64_t s = 0; s < m; s++) {
        sp += nm->x[mem[s]];
        spy += ny(nm, mem[s]);
    }
    for (int64_t s = 0; s < m; s++) {
        int32_t u = mem[s];
        int64_t w_in = 0;
        for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++)
            if (g->col[e] != u && W->part[g->col[e]] == p) w_in += g->w[e];
        const int64_t xu = nm->x[u], yu = ny(nm, u);
        W->gl[u] = nm->A * w_in - (xu * (sp - xu) - yu * (spy - yu));
    }
}

/* Best bisection of one part (Sec. 3.3): returns the key and the cut pair. */
static int64_t best_split(const graph *g, const int32_t *a, const nullm *nm,
                          pwork *W, const int32_t *mem, int64_t m,
                          int32_t *cut1, int32_t *cut2)
{
    int32_t *cycle = xmalloc((size_t)m * sizeof(int32_t));
    int64_t L = part_structure(a, nm, W, mem, m, cycle);
    int32_t p = W->part[mem[0]];
    const int64_t A = nm->A;
    int64_t sp = 0, spy = 0;
    for (int64_t s = 0; s < m; s++) {
        sp += nm->x[mem[s]];
        spy += ny(nm, mem[s]);
    }

    int have = 0;
    int64_t best = 0;
    int32_t b1 = -1, b2 = -1;
#define CONSIDER(KEY, F, S)                                                    \
    do {                                                                       \
        int64_t key_ = (KEY);                                                  \
        int32_t f_ = (F), s_ = (S);                                            \
        if (!have || key_ > best ||                                            \
            (key_ == best && (f_ < b1 || (f_ == b1 && s_ < b2)))) {            \
            have = 1;                                                          \
            best = key_;                                                       \
            b1 = f_;                                                           \
            b2 = s_;                                                           \
        }                                                                      \
    } while (0)

    /* branch cuts: remove the assignment of a non-cycle node x; one side is
     * the subtree T_x (x and every node whose path passes through x) */
    for (int64_t s = 0; s < m; s++) {
        int32_t x = mem[s];
        if (W->cyc[x]) continue;
        int64_t cut = 0;
        for (int32_t t = W->tin[x]; t < W->tout[x]; t++) {
            int32_t u = W->order[t];
            for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++) {
                int32_t v = g->col[e];
                if (W->part[v] != p) continue;
                int in_tx = W->tin[v] >= W->tin[x] && W->tin[v] < W->tout[x];
                if (!in_tx) cut += g->w[e];
            }
        }
        int64_t s1 = W->sub[x], t1 = W->suby[x];
        CONSIDER(s1 * (sp - s1) - t1 * (spy - t1) - A * cut, x, x);
    }
    /* cycle cuts: remove the assignments of two cycle nodes c_p and c_q
     * (p < q); the side rooted at c_q holds the hanging trees of cycle
     * positions p+1..q, the other side the rest */
    for (int64_t pp = 0; pp < L; pp++) {
        for (int64_t qq = pp + 1; qq < L; qq++) {
            int64_t sy = 0, ty = 0, cut = 0;
            for (int64_t s = 0; s < m; s++) {
                int32_t u = mem[s];
                int in_y = W->pos[u] > pp && W->pos[u] <= qq;
                if (!in_y) continue;
                sy += nm->x[u];
                ty += ny(nm, u);
                for (int64_t e = g->rp[u]; e < g->rp[u + 1]; e++) {
                    int32_t v = g->col[e];
                    if (W->part[v] != p) continue;
                    int v_in_y = W->pos[v] > pp && W->pos[v] <= qq;
                    if (!v_in_y) cut += g->w[e];
                }
            }
            int32_t x = cycle[pp], y = cycle[qq];
            int32_t f = x < y ? x : y, sc = x < y ? y : x;
            CONSIDER(sy * (sp - sy) - ty * (spy - ty) - A * cut, f, sc);
        }
    }
#undef CONSIDER
    free(cycle);
    *cut1 = b1;
    *cut2 = b2;
    return best;
}

/* Gathers the members of the part containing node s into mem (by following
 * the assignment graph in both directions); returns the member count. */
static int64_t gather_part(const int32_t *a, const int32_t *rev_head,
                           const int32_t *rev_next, int32_t *mark, int32_t stamp,
                           int32_t s, int32_t *mem)
{
    int64_t m = 0;
    mem[m++] = s;
    mark[s] = stamp;
    for (int64_t q = 0; q < m; q++) {
        int32_t u = mem[q];
        int32_t v = a[u];
        if (mark[v] != stamp) {
            mark[v] = stamp;
            mem[m++] = v;
        }
        for (int32_t c = rev_head[u]; c >= 0; c = rev_next[c]) {
            if (mark[c] != stamp) {
                mark[c] = stamp;
                mem[m++] = c;
            }
        }
    }
    return m;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Runs POSITIVE on the assignment `a` (modified in place); returns the
 * number of splits applied.  Parts are processed from a work list; every
 * part is split once per visit and both sides go back on the list, which
 * is the per-community loop of the appendix POSITIVE (communities are
 * independent, so the order of visits does not change the result). */
int64_t or_positive_nm(int64_t n, const int64_t *rp, const int32_t *col,
                       const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                       int32_t *a)
{
    graph g = {n, rp, col, w};
    const nullm nm = {x, y, A};
    pwork W;
    W.n = n;
    W.part = xmalloc((size_t)n * sizeof(int32_t));
    W.cyc = xcalloc((size_t)n, 1);
    W.tin = xmalloc((size_t)n * sizeof(int32_t));
    W.tout = xmalloc((size_t)n * sizeof(int32_t));
    W.order = xmalloc((size_t)n * sizeof(int32_t));
    W.pos = xmalloc((size_t)n * sizeof(int32_t));
    W.head = xmalloc((size_t)n * sizeof(int32_t));
    W.next = xmalloc((size_t)n * sizeof(int32_t));
    W.sub = xmalloc((size_t)n * sizeof(int64_t));
    W.suby = xmalloc((size_t)n * sizeof(int64_t));
    W.gl = xmalloc((size_t)n * sizeof(int64_t));
    int32_t *rev_head = xmalloc((size_t)n * sizeof(int32_t));
    int32_t *rev_next = xmalloc((size_t)n * sizeof(int32_t));
    int32_t *mark = xmalloc((size_t)n * sizeof(int32_t));
    int32_t *mem = xmalloc((size_t)n * sizeof(int32_t));
    int32_t *work = xmalloc((size_t)(n + 1) * sizeof(int32_t));

    /* initial parts = components of the assignment graph */
    int32_t *lab = xmalloc((size_t)n * sizeof(int32_t));
    int64_t nparts = or_components(n, a, lab, NULL);
    for (int64_t i = 0; i < n; i++) {
        W.part[i] = lab[i];
        mark[i] = -1;
    }
    free(lab);
    /* reverse pointers of T (children and cycle predecessors) */
    for (int64_t i = 0; i < n; i++) rev_head[i] = -1;
    for (int64_t i = n - 1; i >= 0; i--) {
        if (a[i] == i) continue;
        rev_next[i] = rev_head[a[i]];
        rev_head[a[i]] = (int32_t)i;
    }
    /* the smallest member of every part seeds the work list */
    int64_t top = 0;
    {
        uint8_t *seen = xcalloc((size_t)(nparts ? nparts : 1), 1);
        for (int64_t i = 0; i < n; i++)
            if (!seen[W.part[i]]) {
                seen[W.part[i]] = 1;
                work[top++] = (int32_t)i;
            }
        free(seen);
    }
    int32_t stamp = 0;
    int64_t splits = 0;
    int32_t next_part = (int32_t)nparts;
    while (top > 0) {
        int32_t seed = work[--top];
        int64_t m = gather_part(a, rev_head, rev_next, mark, stamp++, seed, mem);
        qsort(mem, (size_t)m, sizeof(int32_t), cmp_i32);
        int32_t pid = next_part++;
        for (int64_t s = 0; s < m; s++) W.part[mem[s]] = pid;
        part_gains(&g, &nm, &W, mem, m);
        int negative = 0;
        for (int64_t s = 0; s < m; s++)
            if (W.gl[mem[s]] < 0) negative = 1;
        if (!negative) continue;
        int32_t cx, cy;
        best_split(&g, a, &nm, &W, mem, m, &cx, &cy);
        /* the two sides: a branch cut separates T_x from the part of x's old
         * target; a cycle cut separates the sides rooted at x and at y */
        int32_t seed_a = cx, seed_b = (cx == cy) ? a[cx] : cy;
        int32_t cut_nodes[2] = {cx, cy};
        for (int c = 0; c < (cx == cy ? 1 : 2); c++) {
            int32_t u = cut_nodes[c];
            int32_t *link = &rev_head[a[u]];
            while (*link != u) link = &rev_next[*link];
            *link = rev_next[u];
            a[u] = u; /* the removed assignment becomes a self-assignment */
        }
        splits++;
        work[top++] = seed_b;
        work[top++] = seed_a;
    }
    free(work);
    free(mem);
    free(mark);
    free(rev_next);
    free(rev_head);
    free(W.gl);
    free(W.suby);
    free(W.sub);
    free(W.next);
    free(W.head);
    free(W.pos);
    free(W.order);
    free(W.tout);
    free(W.tin);
    free(W.cyc);
    free(W.part);
    return splits;
}

int64_t or_positive(int64_t n, const int64_t *rp, const int32_t *col,
                    const int32_t *w, const int64_t *k, int64_t m2, int32_t *a)
{
    return or_positive_nm(n, rp, col, w, k, NULL, m2, a);
}

/* ------------------------------------------------------------------------ */
/* MAXIMAL (Sec. 3.4, appendix MAXIMAL).                                     */
/* ------------------------------------------------------------------------ */

/* The first loop of MAXIMAL: every node's best community, all computed from
 * the same labelling.  best_c[i] = argmax_C join(i,C) over neighbouring
 * communities C != c_i (ties to the lowest label) when that beats stay(i),
 * else c_i; delta[i] = join - stay for a move and 0 otherwise; w_own[i] =
 * w(i, c_i \ i).  A dense accumulator with a touched list totals w(i,C). */
void or_sweep_nm(int64_t n, const int64_t *rp, const int32_t *col,
                 const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                 const int32_t *lab, int64_t nc, int32_t *best_c, int64_t *delta,
                 int32_t *w_own)
{
    const nullm nm = {x, y, A};
    int64_t *sig = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    int64_t *sgy = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    null_totals(n, &nm, lab, nc, sig, sgy);
    int64_t *acc = xcalloc((size_t)(nc ? nc : 1), sizeof(int64_t));
    int32_t *touched = xmalloc((size_t)(nc ? nc : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) {
        int64_t nt = 0, w_in = 0;
        int32_t ci = lab[i];
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int32_t v = col[e];
            if (v == i) continue;
            if (lab[v] == ci) {
                w_in += w[e];
                continue;
            }
            if (acc[lab[v]] == 0) touched[nt++] = lab[v];
            acc[lab[v]] += w[e];
        }
        const int64_t xi = x[i], yi = ny(&nm, i);
        int64_t stay = A * w_in - (xi * (sig[ci] - xi) - yi * (sgy[ci] - yi));
        int64_t best_key = 0;
        int32_t best = -1;
        for (int64_t t = 0; t < nt; t++) {
            int32_t c = touched[t];
            int64_t key = A * acc[c] - (xi * sig[c] - yi * sgy[c]);
            if (best < 0 || key > best_key || (key == best_key && c < best)) {
                best = c;
                best_key = key;
            }
            acc[c] = 0;
        }
        if (best >= 0 && best_key > stay) {
            best_c[i] = best;
            delta[i] = best_key - stay;
        } else {
            best_c[i] = ci;
            delta[i] = 0;
        }
        w_own[i] = (int32_t)w_in;
    }
    free(touched);
    free(acc);
    free(sgy);
    free(sig);
}

void or_sweep(int64_t n, const int64_t *rp, const int32_t *col,
              const int32_t *w, const int64_t *k, int64_t m2,
              const int32_t *lab, int64_t nc, int32_t *best_c, int64_t *delta,
              int32_t *w_own)
{
    or_sweep_nm(n, rp, col, w, k, NULL, m2, lab, nc, best_c, delta, w_own);
}

/* Forest view of an assignment graph: cycle nodes are roots, every other
 * node's parent is a(u).  DFS times make every subtree a contiguous range of
 * `order`; the members of each community are listed by label. */
typedef struct {
    uint8_t *cyc;
    int32_t *tin, *tout, *order;
    int64_t *mem_off; /* members of community c: mem[mem_off[c] .. mem_off[c+1]) */
    int32_t *mem;
} forest;

static void build_forest(int64_t n, const int32_t *a, const int32_t *lab,
                         int64_t nc, forest *F)
{
    F->cyc = xmalloc((size_t)n);
    F->tin = xmalloc((size_t)n * sizeof(int32_t));
    F->tout = xmalloc((size_t)n * sizeof(int32_t));
    F->order = xmalloc((size_t)n * sizeof(int32_t));
    F->mem_off = xcalloc((size_t)nc + 1, sizeof(int64_t));
    F->mem = xmalloc((size_t)n * sizeof(int32_t));
    int32_t *tmp = xmalloc((size_t)n * sizeof(int32_t));
    or_components(n, a, tmp, F->cyc);
    free(tmp);
    for (int64_t i = 0; i < n; i++) F->mem_off[lab[i] + 1]++;
    for (int64_t c = 0; c < nc; c++) F->mem_off[c + 1] += F->mem_off[c];
    int64_t *fill = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    for (int64_t c = 0; c < nc; c++) fill[c] = F->mem_off[c];
    for (int64_t i = 0; i < n; i++) F->mem[fill[lab[i]]++] = (int32_t)i;
    free(fill);
    /* children lists in increasing id order, then one DFS per cycle node */
    int32_t *head = xmalloc((size_t)n * sizeof(int32_t));
    int32_t *next = xmalloc((size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) head[i] = -1;
    for (int64_t i = n - 1; i >= 0; i--) {
        if (F->cyc[i]) continue;
        next[i] = head[a[i]];
        head[a[i]] = (int32_t)i;
    }
    int32_t *stack = xmalloc((size_t)n * sizeof(int32_t));
    int64_t t = 0;
    for (int64_t r = 0; r < n; r++) {
        if (!F->cyc[r]) continue;
        int64_t sp = 0;
        stack[sp++] = (int32_t)r;
        F->tin[r] = (int32_t)t;
        F->order[t++] = (int32_t)r;
        while (sp > 0) {
            int32_t u = stack[sp - 1];
            int32_t c = head[u];
            if (c >= 0) {
                head[u] = next[c];
                F->tin[c] = (int32_t)t;
                F->order[t++] = c;
                stack[sp++] = c;
            } else {
                F->tout[u] = (int32_t)t;
                sp--;
            }
        }
    }
    free(stack);
    free(next);
    free(head);
}

static void free_forest(forest *F)
{
    free(F->cyc);
    free(F->tin);
    free(F->tout);
    free(F->order);
    free(F->mem_off);
    free(F->mem);
}

/* One correction round of MAXIMAL followed by POSITIVE (the body of the inner
 * loop of Algorithm 1).  For every node whose best community differs from its
 * own, the tail B (the node and every node with a path to it; the whole
 * community when the node is on the cycle) is checked: the move is valid iff
 * move(B: c -> c*) > 0.  When no node is valid the round changes nothing and
 * returns 0.  Otherwise every valid node draws; an accepted node i re-points
 * a(i) to its best neighbour inside c_i* (largest pair(i,j), ties to the
 * lowest j).  All re-pointings use the state before the round and are
 * applied together; the communities then are the components of the new
 * assignment graph, and POSITIVE runs on them.
 * stats (optional, 4 entries): candidates, valid, accepted, splits. */
int64_t or_maximal_round_nm(int64_t n, const int64_t *rp, const int32_t *col,
                            const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                            int32_t *a, uint64_t seed, int32_t level, int32_t round,
                            uint64_t accept_p, int64_t *stats, int32_t *a_repointed);

int64_t or_maximal_round(int64_t n, const int64_t *rp, const int32_t *col,
                         const int32_t *w, const int64_t *k, int64_t m2,
                         int32_t *a, uint64_t seed, int32_t level, int32_t round,
                         uint64_t accept_p, int64_t *stats)
{
    return or_maximal_round_nm(n, rp, col, w, k, NULL, m2, a, seed, level, round, accept_p,
                               stats, NULL);
}

/* As or_maximal_round; a_repointed (optional) receives the assignment after
 * the re-pointing and before POSITIVE (unchanged when no move is valid). */
int64_t or_maximal_round_ex(int64_t n, const int64_t *rp, const int32_t *col,
                            const int32_t *w, const int64_t *k, int64_t m2,
                            int32_t *a, uint64_t seed, int32_t level, int32_t round,
                            uint64_t accept_p, int64_t *stats, int32_t *a_repointed)
{
    return or_maximal_round_nm(n, rp, col, w, k, NULL, m2, a, seed, level, round, accept_p,
                               stats, a_repointed);
}

/* The round under any null model (x, y, A); see nullm. */
int64_t or_maximal_round_nm(int64_t n, const int64_t *rp, const int32_t *col,
                            const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                            int32_t *a, uint64_t seed, int32_t level, int32_t round,
                            uint64_t accept_p, int64_t *stats, int32_t *a_repointed)
{
    const nullm nm = {x, y, A};
    int32_t *lab = xmalloc((size_t)n * sizeof(int32_t));
    int64_t nc = or_components(n, a, lab, NULL);
    int64_t *sig = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    int64_t *sgy = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    null_totals(n, &nm, lab, nc, sig, sgy);
    int32_t *best_c = xmalloc((size_t)n * sizeof(int32_t));
    int64_t *delta = xmalloc((size_t)n * sizeof(int64_t));
    int32_t *w_own = xmalloc((size_t)n * sizeof(int32_t));
    or_sweep_nm(n, rp, col, w, x, y, A, lab, nc, best_c, delta, w_own);

    forest F;
    build_forest(n, a, lab, nc, &F);
    uint8_t *accepted = xcalloc((size_t)n, 1);
    int64_t n_cand = 0, n_valid = 0, n_acc = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t c = lab[i], d = best_c[i];
        if (d == c) continue;
        n_cand++;
        /* members of the tail B */
        const int32_t *bm;
        int64_t bcount;
        if (F.cyc[i]) {
            bm = F.mem + F.mem_off[c];
            bcount = F.mem_off[c + 1] - F.mem_off[c];
        } else {
            bm = F.order + F.tin[i];
            bcount = F.tout[i] - F.tin[i];
        }
        int64_t sb = 0, tb = 0, w_bd = 0, w_brest = 0;
        for (int64_t s = 0; s < bcount; s++) {
            int32_t u = bm[s];
            sb += x[u];
            tb += ny(&nm, u);
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
                int32_t v = col[e];
                if (lab[v] == d) w_bd += w[e];
                else if (lab[v] == c) {
                    int v_in_b = F.cyc[i] ? 1 : (F.tin[v] >= F.tin[i] && F.tin[v] < F.tout[i]);
                    if (!v_in_b) w_brest += w[e];
                }
            }
        }
        int64_t mv = A * (w_bd - w_brest) -
                     (sb * (sig[d] - sig[c] + sb) - tb * (sgy[d] - sgy[c] + tb));
        if (mv <= 0) continue;
        n_valid++;
        if ((uint64_t)or_draw(seed, level, round, (int32_t)i) < accept_p) {
            accepted[i] = 1;
            n_acc++;
        }
    }
    free_forest(&F);
    int64_t splits = 0;
    if (n_valid > 0) {
        /* re-point every accepted node, reading only the pre-round state */
        int32_t *a_new = xmalloc((size_t)n * sizeof(int32_t));
        memcpy(a_new, a, (size_t)n * sizeof(int32_t));
        for (int64_t i = 0; i < n; i++) {
            if (!accepted[i]) continue;
            int32_t d = best_c[i];
            int64_t best_j = -1, best_key = 0;
            for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
                int64_t j = col[e];
                if (lab[j] != d) continue;
                int64_t key = A * (int64_t)w[e] - (x[i] * x[j] - ny(&nm, i) * ny(&nm, j));
                if (best_j < 0 || key > best_key || (key == best_key && j < best_j)) {
                    best_j = j;
                    best_key = key;
                }
            }
            a_new[i] = (int32_t)best_j;
        }
        memcpy(a, a_new, (size_t)n * sizeof(int32_t));
        free(a_new);
        if (a_repointed) memcpy(a_repointed, a, (size_t)n * sizeof(int32_t));
        splits = or_positive_nm(n, rp, col, w, x, y, A, a);
    } else if (a_repointed) {
        memcpy(a_repointed, a, (size_t)n * sizeof(int32_t));
    }
    if (stats) {
        stats[0] = n_cand;
        stats[1] = n_valid;
        stats[2] = n_acc;
        stats[3] = splits;
    }
    free(accepted);
    free(w_own);
    free(delta);
    free(best_c);
    free(sgy);
    free(sig);
    free(lab);
    return n_valid;
}

/* ------------------------------------------------------------------------ */
/* Modularity (Sec. 2.4, weighted form with m_w = M2):                       */
/*   N_Q = M2 * sum_C w(C,C) - sum_C S_C^2,   Q = N_Q / M2^2.                */
/* ------------------------------------------------------------------------ */

int64_t or_modularity_num_nm(int64_t n, const int64_t *rp, const int32_t *col,
                             const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                             const int32_t *lab, int64_t nc)
{
    const nullm nm = {x, y, A};
    int64_t *sig = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    int64_t *sgy = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    null_totals(n, &nm, lab, nc, sig, sgy);
    int64_t inside = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rp[i]; e < rp[i + 1]; e++)
            if (lab[col[e]] == lab[i]) inside += w[e];
    int64_t sq = 0;
    for (int64_t c = 0; c < nc; c++) sq += sig[c] * sig[c] - sgy[c] * sgy[c];
    free(sgy);
    free(sig);
    return A * inside - sq;
}

int64_t or_modularity_num(int64_t n, const int64_t *rp, const int32_t *col,
                          const int32_t *w, const int64_t *k, int64_t m2,
                          const int32_t *lab, int64_t nc)
{
    return or_modularity_num_nm(n, rp, col, w, k, NULL, m2, lab, nc);
}

double or_modularity(int64_t nq, int64_t m2)
{
    if (m2 == 0) return 0.0;
    return (double)nq / (double)m2 / (double)m2;
}

/* ------------------------------------------------------------------------ */
/* AGGREGATE (Sec. 3.5): communities become the nodes of the next level;     */
/* A'_CD = sum of A_uv over u in C, v in D (diagonal included).              */
/* Output rows are sorted by column.  Returns the new entry count.           */
/* ------------------------------------------------------------------------ */

int64_t or_contract(int64_t n, const int64_t *rp, const int32_t *col,
                    const int32_t *w, const int32_t *lab, int64_t nc,
                    int64_t *rp_out, int32_t *col_out, int32_t *w_out)
{
    /* members by community */
    int64_t *off = xcalloc((size_t)nc + 1, sizeof(int64_t));
    int32_t *mem = xmalloc((size_t)(n ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) off[lab[i] + 1]++;
    for (int64_t c = 0; c < nc; c++) off[c + 1] += off[c];
    int64_t *fill = xmalloc((size_t)(nc ? nc : 1) * sizeof(int64_t));
    for (int64_t c = 0; c < nc; c++) fill[c] = off[c];
    for (int64_t i = 0; i < n; i++) mem[fill[lab[i]]++] = (int32_t)i;
    free(fill);
    int64_t *acc = xcalloc((size_t)(nc ? nc : 1), sizeof(int64_t));
    int32_t *touched = xmalloc((size_t)(nc ? nc : 1) * sizeof(int32_t));
    int64_t out = 0;
    rp_out[0] = 0;
    for (int64_t c = 0; c < nc; c++) {
        int64_t nt = 0;
        for (int64_t s = off[c]; s < off[c + 1]; s++) {
            int32_t u = mem[s];
            for (int64_t e = rp[u]; e < rp[u + 1]; e++) {
                int32_t d = lab[col[e]];
                if (acc[d] == 0) touched[nt++] = d;
                acc[d] += w[e];
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < nt; t++) {
            col_out[out] = touched[t];
            w_out[out] = (int32_t)acc[touched[t]];
            acc[touched[t]] = 0;
            out++;
        }
        rp_out[c + 1] = out;
    }
    free(touched);
    free(acc);
    free(mem);
    free(off);
    return out;
}

/* ------------------------------------------------------------------------ */
/* Level loop (Algorithm 1).                                                 */
/* ------------------------------------------------------------------------ */

/* One level: ASSIGN, POSITIVE, then MAXIMAL+POSITIVE rounds until no valid
 * move is left or max_rounds rounds have applied moves.  Writes the final
 * assignment; returns the number of rounds that applied moves, and sets
 * *converged to 1 when the loop ended because no move was valid. */
int32_t or_level_nm(int64_t n, const int64_t *rp, const int32_t *col,
                    const int32_t *w, const int64_t *x, const int64_t *y, int64_t A,
                    uint64_t seed, int32_t level, uint64_t accept_p, int32_t max_rounds,
                    int32_t *a, int32_t *converged, int64_t *totals)
{
    or_assign_nm(n, rp, col, w, x, y, A, a);
    int64_t splits = or_positive_nm(n, rp, col, w, x, y, A, a);
    int32_t r = 0;
    *converged = 0;
    int64_t st[4], tot_acc = 0, tot_valid = 0;
    while (r < max_rounds) {
        int64_t valid = or_maximal_round_nm(n, rp, col, w, x, y, A, a, seed, level, r,
                                            accept_p, st, NULL);
        if (valid == 0) {
            *converged = 1;
            break;
        }
        tot_valid += st[1];
        tot_acc += st[2];
        splits += st[3];
        if (getenv("SLM_ORACLE_VERBOSE"))
            fprintf(stderr, "oracle level %d round %d: candidates %lld valid %lld "
                    "accepted %lld splits %lld\n", level, r, (long long)st[0],
                    (long long)st[1], (long long)st[2], (long long)st[3]);
        r++;
    }
    if (totals) {
        totals[0] = tot_valid;
        totals[1] = tot_acc;
        totals[2] = splits;
    }
    return r;
}

int32_t or_level(int64_t n, const int64_t *rp, const int32_t *col,
                 const int32_t *w, const int64_t *k, int64_t m2, uint64_t seed,
                 int32_t level, uint64_t accept_p, int32_t max_rounds,
                 int32_t *a, int32_t *converged, int64_t *totals)
{
    return or_level_nm(n, rp, col, w, k, NULL, m2, seed, level, accept_p, max_rounds, a,
                       converged, totals);
}

/* Full run of Algorithm 1.  Levels whose partition is the identity are not
 * emitted and end the run.  For every emitted level l (at most max_out):
 * labels_out[l*n0 .. (l+1)*n0) = community of every original node (the
 * composition of all levels so far), nc_out[l], nq_out[l], q_out[l],
 * rounds_out[l], conv_out[l].  Returns the number of emitted levels. */
int32_t or_run(int64_t n0, const int64_t *rp0, const int32_t *col0,
               const int32_t *w0, uint64_t seed, uint64_t accept_p,
               int32_t max_rounds, int32_t max_levels, int32_t max_out,
               int32_t *labels_out, int64_t *nc_out, int64_t *nq_out,
               double *q_out, int32_t *rounds_out, int32_t *conv_out)
{
    int64_t nnz0 = rp0[n0];
    int64_t n = n0;
    int64_t *rp = xmalloc((size_t)(n0 + 1) * sizeof(int64_t));
    int32_t *col = xmalloc((size_t)(nnz0 ? nnz0 : 1) * sizeof(int32_t));
    int32_t *w = xmalloc((size_t)(nnz0 ? nnz0 : 1) * sizeof(int32_t));
    memcpy(rp, rp0, (size_t)(n0 + 1) * sizeof(int64_t));
    memcpy(col, col0, (size_t)nnz0 * sizeof(int32_t));
    memcpy(w, w0, (size_t)nnz0 * sizeof(int32_t));
    int64_t *k = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int64_t));
    int32_t *a = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    int32_t *lab = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    int32_t *composed = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    for (int64_t v = 0; v < n0; v++) composed[v] = (int32_t)v;
    int64_t m2 = or_strength(n, rp, col, w, k);
    int32_t emitted = 0;
    int32_t level = 0;
    while (m2 > 0 && n > 0) {
        int32_t conv = 0;
        int32_t rounds = or_level(n, rp, col, w, k, m2, seed, level, accept_p,
                                  max_rounds, a, &conv, NULL);
        int64_t nc = or_components(n, a, lab, NULL);
        if (nc == n) break; /* the level partition is the identity */
        for (int64_t v = 0; v < n0; v++) composed[v] = lab[composed[v]];
        int64_t nq = or_modularity_num(n, rp, col, w, k, m2, lab, nc);
        if (emitted < max_out) {
            memcpy(labels_out + (size_t)emitted * (size_t)n0, composed,
                   (size_t)n0 * sizeof(int32_t));
            nc_out[emitted] = nc;
            nq_out[emitted] = nq;
            q_out[emitted] = or_modularity(nq, m2);
            rounds_out[emitted] = rounds;
            conv_out[emitted] = conv;
        }
        emitted++;
        /* next level */
        int64_t nnz = rp[n];
        int64_t *rp2 = xmalloc((size_t)(nc + 1) * sizeof(int64_t));
        int32_t *col2 = xmalloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
        int32_t *w2 = xmalloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
        or_contract(n, rp, col, w, lab, nc, rp2, col2, w2);
        free(rp);
        free(col);
        free(w);
        rp = rp2;
        col = col2;
        w = w2;
        n = nc;
        or_strength(n, rp, col, w, k);
        level++;
        if (max_levels > 0 && emitted >= max_levels) break;
    }
    free(composed);
    free(lab);
    free(a);
    free(k);
    free(w);
    free(col);
    free(rp);
    return emitted;
}

/* ------------------------------------------------------------------------ */
/* Null models (Sec. 2.2-2.4).  A model is (kind, num, den):                */
/*   kind 0, configuration model of an undirected graph with resolution     */
/*     gamma = num/den: the modularity of Sec. 2.4 with the null-model term  */
/*     scaled by gamma; x = num*k, y = 0, A = num*den*M2 (gains are num      */
/*     times M2*den*w - gamma*den*... i.e. a positive multiple).             */
/*   kind 1, Erdos-Renyi null model of Sec. 2.3 with p_ij = p = num/den:    */
/*     the energy of Sec. 2.2 with alpha = 1 and beta = p for every pair;    */
/*     x = num*size (size = original nodes a node stands for, 1 at level 0), */
/*     y = 0, A = num*den.                                                   */
/*   kind 2, configuration model of a directed graph W (Sec. 2.4 with out-  */
/*     and in-strengths), resolution gamma = num/den: the level runs on the  */
/*     symmetric S = W + W^T, x = num*(k_out + k_in), y = num*(k_out - k_in), */
/*     A = num*den*sum(S).  Merging P and R changes                          */
/*     sum_ij [den*m*W_ij - num*k_out_i*k_in_j] over pairs in one community  */
/*     by (A*S(P,R) - X_P X_R + Y_P Y_R) / (2 num), m = sum(W).              */
/* (0, 1, 1) is the default model, x = k and A = M2.  The modularity value   */
/* reported is Q = N_Q / A / M2 with N_Q = A*sum_C S(C,C) - sum_C (X^2-Y^2)  */
/* and M2 = sum(S).                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t r, c, w;
} triple;

static int cmp_triple(const void *p, const void *q)
{
    const triple *a = p, *b = q;
    if (a->r != b->r) return (a->r > b->r) - (a->r < b->r);
    return (a->c > b->c) - (a->c < b->c);
}

/* S = W + W^T as a CSR with sorted columns (diagonal entries become 2 W_ii).
 * rp_out: n+1, col_out and w_out: up to 2 nnz entries.  Returns nnz(S). */
int64_t or_symmetrize(int64_t n, const int64_t *rp, const int32_t *col, const int32_t *w,
                      int64_t *rp_out, int32_t *col_out, int32_t *w_out)
{
    int64_t nnz = rp[n];
    triple *t = xmalloc((size_t)(2 * nnz) * sizeof(triple));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            t[m++] = (triple){i, col[e], w[e]};
            t[m++] = (triple){col[e], i, w[e]};
        }
    qsort(t, (size_t)m, sizeof(triple), cmp_triple);
    int64_t out = 0;
    for (int64_t i = 0; i <= n; i++) rp_out[i] = 0;
    for (int64_t s = 0; s < m; s++) {
        if (out > 0 && s > 0 && t[s].r == t[s - 1].r && t[s].c == t[s - 1].c) {
            w_out[out - 1] += (int32_t)t[s].w;
            continue;
        }
        col_out[out] = (int32_t)t[s].c;
        w_out[out] = (int32_t)t[s].w;
        rp_out[t[s].r + 1]++;
        out++;
    }
    for (int64_t i = 0; i < n; i++) rp_out[i + 1] += rp_out[i];
    free(t);
    return out;
}

#define OR_BOUND ((int64_t)1 << 61)

/* Strengths of a model on the level-0 graph (rp, col, w): for kind 2 that is
 * the directed W, and (srp, scol, sw) must hold S = W + W^T.  Writes x, y
 * (n each), *A and *M2 (sum of the matrix the levels run on).  Returns 0,
 * 1 for an invalid model, 2 when the gains could leave int64 (A*M2 or
 * sum(x)^2 above 2^61; the default model keeps its own M2 < 2^31 bound). */
int32_t or_null_strengths(int32_t kind, int64_t num, int64_t den, int64_t n,
                          const int64_t *rp, const int32_t *col, const int32_t *w,
                          int64_t *x, int64_t *y, int64_t *A_out, int64_t *M2_out)
{
    if (num < 1 || den < 1 || kind < 0 || kind > 2) return 1;
    int64_t m2 = 0;
    for (int64_t i = 0; i < n; i++) {
        x[i] = 0;
        y[i] = 0;
    }
    for (int64_t i = 0; i < n; i++)
        for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
            int64_t v = w[e];
            m2 += v;
            if (kind == 2) {
                x[i] += v;      /* k_out(i) */
                x[col[e]] += v; /* k_in(col) */
                y[i] += v;
                y[col[e]] -= v;
            } else {
                x[i] += v;
            }
        }
    if (kind == 2) m2 *= 2; /* sum of S = W + W^T */
    if (m2 >= ((int64_t)1 << 31)) return 2;
    const int default_model = kind == 0 && num == 1 && den == 1;
    if (!default_model && num > ((int64_t)1 << 30)) return 2;
    int64_t xt = 0;
    for (int64_t i = 0; i < n; i++) {
        if (kind == 1) x[i] = 1;
        x[i] *= num;
        y[i] *= num;
        xt += x[i];
    }
    const int64_t base = kind == 1 ? 1 : m2;
    if (!default_model) {
        /* every gain then stays within 2^62 in magnitude */
        if (xt > ((int64_t)1 << 30)) return 2;
        if (num > OR_BOUND / den) return 2;
        const int64_t nd = num * den;
        if (base > 0 && nd > OR_BOUND / base) return 2;
        if (m2 > 0 && nd * base > OR_BOUND / m2) return 2;
    }
    *A_out = num * den * base;
    *M2_out = m2;
    return 0;
}

double or_modularity_nm(int64_t nq, int64_t A, int64_t m2)
{
    if (A == 0 || m2 == 0) return 0.0;
    return (double)nq / (double)A / (double)m2;
}

/* Full run under a null model (see above): the input is symmetric for kinds
 * 0 and 1 and any CSR W for kind 2.  Levels run on S (kind 2) or the input;
 * x and y of a community are the sums over its members at every
 * contraction.  Outputs as or_run; returns the emitted level count, or -1
 * (invalid model) / -2 (bounds). */
int32_t or_run_null(int64_t n0, const int64_t *rp0, const int32_t *col0,
                    const int32_t *w0, int32_t kind, int64_t num, int64_t den,
                    uint64_t seed, uint64_t accept_p, int32_t max_rounds,
                    int32_t max_levels, int32_t max_out, int32_t *labels_out,
                    int64_t *nc_out, int64_t *nq_out, double *q_out,
                    int32_t *rounds_out, int32_t *conv_out)
{
    int64_t nnz0 = rp0[n0];
    int64_t cap = kind == 2 ? 2 * nnz0 : nnz0;
    int64_t n = n0;
    int64_t *rp = xmalloc((size_t)(n0 + 1) * sizeof(int64_t));
    int32_t *col = xmalloc((size_t)(cap ? cap : 1) * sizeof(int32_t));
    int32_t *w = xmalloc((size_t)(cap ? cap : 1) * sizeof(int32_t));
    int64_t *x = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int64_t));
    int64_t *y = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int64_t));
    int64_t A = 0, m2 = 0;
    int32_t st = or_null_strengths(kind, num, den, n0, rp0, col0, w0, x, y, &A, &m2);
    if (st != 0) {
        free(y);
        free(x);
        free(w);
        free(col);
        free(rp);
        return st == 1 ? -1 : -2;
    }
    int64_t nnz;
    if (kind == 2) {
        nnz = or_symmetrize(n0, rp0, col0, w0, rp, col, w);
    } else {
        nnz = nnz0;
        memcpy(rp, rp0, (size_t)(n0 + 1) * sizeof(int64_t));
        memcpy(col, col0, (size_t)nnz0 * sizeof(int32_t));
        memcpy(w, w0, (size_t)nnz0 * sizeof(int32_t));
    }
    (void)nnz;
    const int64_t *yy = kind == 2 ? y : NULL;
    int32_t *a = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    int32_t *lab = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    int32_t *composed = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    int64_t *tmp = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int64_t));
    for (int64_t v = 0; v < n0; v++) composed[v] = (int32_t)v;
    int32_t emitted = 0;
    int32_t level = 0;
    while (m2 > 0 && n > 0) {
        int32_t conv = 0;
        int32_t rounds = or_level_nm(n, rp, col, w, x, yy, A, seed, level, accept_p,
                                     max_rounds, a, &conv, NULL);
        int64_t nc = or_components(n, a, lab, NULL);
        if (nc == n) break; /* the level partition is the identity */
        for (int64_t v = 0; v < n0; v++) composed[v] = lab[composed[v]];
        int64_t nq = or_modularity_num_nm(n, rp, col, w, x, yy, A, lab, nc);
        if (emitted < max_out) {
            memcpy(labels_out + (size_t)emitted * (size_t)n0, composed,
                   (size_t)n0 * sizeof(int32_t));
            nc_out[emitted] = nc;
            nq_out[emitted] = nq;
            q_out[emitted] = or_modularity_nm(nq, A, m2);
            rounds_out[emitted] = rounds;
            conv_out[emitted] = conv;
        }
        emitted++;
        /* next level: contracted matrix, strengths summed per community */
        int64_t nnz_t = rp[n];
        int64_t *rp2 = xmalloc((size_t)(nc + 1) * sizeof(int64_t));
        int32_t *col2 = xmalloc((size_t)(nnz_t ? nnz_t : 1) * sizeof(int32_t));
        int32_t *w2 = xmalloc((size_t)(nnz_t ? nnz_t : 1) * sizeof(int32_t));
        or_contract(n, rp, col, w, lab, nc, rp2, col2, w2);
        community_totals(n, x, lab, nc, tmp);
        memcpy(x, tmp, (size_t)nc * sizeof(int64_t));
        community_totals(n, y, lab, nc, tmp);
        memcpy(y, tmp, (size_t)nc * sizeof(int64_t));
        free(rp);
        free(col);
        free(w);
        rp = rp2;
        col = col2;
        w = w2;
        n = nc;
        level++;
        if (max_levels > 0 && emitted >= max_levels) break;
    }
    free(tmp);
    free(composed);
    free(lab);
    free(a);
    free(y);
    free(x);
    free(w);
    free(col);
    free(rp);
    return emitted;
}

/* ------------------------------------------------------------------------ */
/* Classical Louvain: the sequential method the SLM is built on, named in    */
/* Sec. 6 as the comparison the paper leaves open.  A level moves nodes one  */
/* at a time, in id order, each to its best neighbouring community with the  */
/* state left by the moves before it (the SLM instead decides every move of  */
/* a round from the same state, Sec. 3.4); passes over all nodes repeat      */
/* until one moves nothing (or max_passes), then AGGREGATE as in Sec. 3.5.   */
/* Same exact keys and ties as the SLM sweep: node i in community c moves to */
/* argmax_{C != c} join(i,C) (lowest C on ties) iff that beats stay(i).      */
/* During a level a community is named by the node it started from, so the  */
/* tie order is that of those ids; the level's labels are then made          */
/* canonical.                                                                */
/* ------------------------------------------------------------------------ */

/* Local moving of one level; lab_out gets the canonical labels.  Returns the
 * community count; *passes = passes that moved a node, *converged = 1 when
 * the last pass moved nothing, *moves = nodes moved in all passes. */
int64_t or_louvain_level(int64_t n, const int64_t *rp, const int32_t *col,
                         const int32_t *w, const int64_t *k, int64_t m2,
                         int32_t max_passes, int32_t *lab_out, int32_t *passes,
                         int32_t *converged, int64_t *moves)
{
    int32_t *c = xmalloc((size_t)(n ? n : 1) * sizeof(int32_t));
    int64_t *sig = xmalloc((size_t)(n ? n : 1) * sizeof(int64_t));
    int64_t *acc = xcalloc((size_t)(n ? n : 1), sizeof(int64_t));
    int32_t *touched = xmalloc((size_t)(n ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) {
        c[i] = (int32_t)i;
        sig[i] = k[i];
    }
    int32_t p = 0;
    int64_t total = 0;
    *converged = 0;
    while (p < max_passes) {
        int64_t moved = 0;
        for (int64_t i = 0; i < n; i++) {
            int32_t ci = c[i];
            int64_t nt = 0, w_in = 0;
            for (int64_t e = rp[i]; e < rp[i + 1]; e++) {
                int32_t v = col[e];
                if (v == i) continue;
                if (c[v] == ci) {
                    w_in += w[e];
                    continue;
                }
                if (acc[c[v]] == 0) touched[nt++] = c[v];
                acc[c[v]] += w[e];
            }
            int64_t stay = m2 * w_in - k[i] * (sig[ci] - k[i]);
            int64_t best_key = 0;
            int32_t best = -1;
            for (int64_t t = 0; t < nt; t++) {
                int32_t cc = touched[t];
                int64_t key = m2 * acc[cc] - k[i] * sig[cc];
                if (best < 0 || key > best_key || (key == best_key && cc < best)) {
                    best = cc;
                    best_key = key;
                }
                acc[cc] = 0;
            }
            if (best >= 0 && best_key > stay) {
                sig[ci] -= k[i];
                sig[best] += k[i];
                c[i] = best;
                moved++;
            }
        }
        if (moved == 0) {
            *converged = 1;
            break;
        }
        total += moved;
        p++;
    }
    /* canonical labels: communities numbered by their smallest member */
    int32_t *name = xmalloc((size_t)(n ? n : 1) * sizeof(int32_t));
    for (int64_t i = 0; i < n; i++) name[i] = -1;
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) {
        if (name[c[i]] < 0) name[c[i]] = (int32_t)nc++;
        lab_out[i] = name[c[i]];
    }
    free(name);
    free(touched);
    free(acc);
    free(sig);
    free(c);
    *passes = p;
    *moves = total;
    return nc;
}

/* Full classical Louvain run: levels until one leaves the identity (not
 * emitted) or max_levels; per emitted level the composed labels, n_c, N_Q,
 * Q (as or_run), the passes that moved nodes and the converged flag. */
int32_t or_louvain_run(int64_t n0, const int64_t *rp0, const int32_t *col0,
                       const int32_t *w0, int32_t max_passes, int32_t max_levels,
                       int32_t max_out, int32_t *labels_out, int64_t *nc_out,
                       int64_t *nq_out, double *q_out, int32_t *passes_out,
                       int32_t *conv_out)
{
    int64_t nnz0 = rp0[n0];
    int64_t n = n0;
    int64_t *rp = xmalloc((size_t)(n0 + 1) * sizeof(int64_t));
    int32_t *col = xmalloc((size_t)(nnz0 ? nnz0 : 1) * sizeof(int32_t));
    int32_t *w = xmalloc((size_t)(nnz0 ? nnz0 : 1) * sizeof(int32_t));
    memcpy(rp, rp0, (size_t)(n0 + 1) * sizeof(int64_t));
    memcpy(col, col0, (size_t)nnz0 * sizeof(int32_t));
    memcpy(w, w0, (size_t)nnz0 * sizeof(int32_t));
    int64_t *k = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int64_t));
    int32_t *lab = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    int32_t *composed = xmalloc((size_t)(n0 ? n0 : 1) * sizeof(int32_t));
    for (int64_t v = 0; v < n0; v++) composed[v] = (int32_t)v;
    int64_t m2 = or_strength(n, rp, col, w, k);
    int32_t emitted = 0;
    while (m2 > 0 && n > 0) {
        int32_t passes = 0, conv = 0;
        int64_t moves = 0;
        int64_t nc = or_louvain_level(n, rp, col, w, k, m2, max_passes, lab, &passes, &conv,
                                      &moves);
        if (nc == n) break;
        for (int64_t v = 0; v < n0; v++) composed[v] = lab[composed[v]];
        int64_t nq = or_modularity_num(n, rp, col, w, k, m2, lab, nc);
        if (emitted < max_out) {
            memcpy(labels_out + (size_t)emitted * (size_t)n0, composed,
                   (size_t)n0 * sizeof(int32_t));
            nc_out[emitted] = nc;
            nq_out[emitted] = nq;
            q_out[emitted] = or_modularity(nq, m2);
            passes_out[emitted] = passes;
            conv_out[emitted] = conv;
        }
        emitted++;
        int64_t nnz = rp[n];
        int64_t *rp2 = xmalloc((size_t)(nc + 1) * sizeof(int64_t));
        int32_t *col2 = xmalloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
        int32_t *w2 = xmalloc((size_t)(nnz ? nnz : 1) * sizeof(int32_t));
        or_contract(n, rp, col, w, lab, nc, rp2, col2, w2);
        free(rp);
        free(col);
        free(w);
        rp = rp2;
        col = col2;
        w = w2;
        n = nc;
        or_strength(n, rp, col, w, k);
        if (max_levels > 0 && emitted >= max_levels) break;
    }
    free(composed);
    free(lab);
    free(k);
    free(w);
    free(col);
    free(rp);
    return emitted;
}
