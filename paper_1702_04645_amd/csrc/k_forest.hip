// Kernels on the assignment graph T = {(i, a(i))} (Sec. 3.2-3.4):
//  - COMPONENTS by pointer doubling: a^(2^K)(i) lies on the cycle of i's
//    component; the minimum along the doubled path gives the cycle minimum,
//    a canonical id of the component; canonical labels rank components by
//    their smallest member.
//  - Forest view: cycle nodes are roots, every other node's parent is a(i).
//    Jump tables J_k = parent^(2^k) give depths, roots, lowest common
//    ancestors, and subtree sums by doubling scatter
//    S_{k+1}(x) = S_k(x) + sum of S_k(y) over y with parent^(2^k)(y) = x.
//  - POSITIVE split keys (branch and cycle cuts) and their application.
//  - MAXIMAL tails: w(B, D) for every candidate through the chain of
//    candidate ancestors, validity, and the acceptance draw.
// Arrays indexed by a community id use node-id space ("comp") during
// POSITIVE and canonical labels elsewhere; kernels take both forms.
#include "slm_forest.h"

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void atomic_max_i64(i64 *p, i64 v)
{
    unsigned long long *q = (unsigned long long *)p;
    unsigned long long old = *q;
    while ((i64)old < v) {
        unsigned long long prev = atomicCAS(q, old, (unsigned long long)v);
        if (prev == old) break;
        old = prev;
    }
}

__device__ __forceinline__ void atomic_min_u64(u64 *p, u64 v)
{
    atomicMin((unsigned long long *)p, (unsigned long long)v);
}

#define NODE_LOOP(n)                                                                  \
    for (i64 u_ = (i64)blockIdx.x * blockDim.x + threadIdx.x; u_ < (n);               \
         u_ += (i64)gridDim.x * blockDim.x)

static unsigned node_grid(i64 n)
{
    i64 g = (n + SLM_BS - 1) / SLM_BS;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// ------------------------------------------------------------------ components
// Pointer doubling over the functional graph a, with (A, M) packed per node
// so that a step gathers one 8-byte pair: A = the node 2^k steps ahead, M =
// the smallest node id among the 2^k nodes from here.
__global__ void k_comp_init(const i32 *__restrict__ a, i64 n, int2 *__restrict__ AM)
{
    NODE_LOOP(n)
    {
        i32 u = (i32)u_, x = a[u];
        AM[u] = make_int2(x, u < x ? u : x);
    }
}

// One doubling step.  A step that changes nothing leaves both buffers equal
// to the final state (A maps every node onto a cycle whose length divides
// the steps taken, and M of a cycle node covers its cycle), so the steps
// after it return at once: step k runs only if step k-1 set prev_changed.
__global__ void k_comp_step(const int2 *__restrict__ Ii, int2 *__restrict__ Io, i64 n,
                            const int *__restrict__ prev_changed, int *__restrict__ changed)
{
    if (prev_changed && *prev_changed == 0) return;
    bool ch = false;
    NODE_LOOP(n)
    {
        const int2 p = Ii[u_];
        const int2 q = Ii[p.x];
        Io[u_] = make_int2(q.x, p.y < q.y ? p.y : q.y);
        ch |= q.x != p.x || q.y < p.y;
    }
    if (__ballot(ch) != 0 && (threadIdx.x & 63) == 0) *changed = 1;
}

// cmin[u] = the minimum of u's cycle; cyc marks the image of A = cycle nodes.
__global__ void k_comp_mark(const int2 *__restrict__ AM, i64 n, i32 *__restrict__ cmin,
                            uint8_t *__restrict__ cyc)
{
    NODE_LOOP(n)
    {
        const i32 z = AM[u_].x;
        cmin[u_] = AM[z].y;
        cyc[z] = 1;
    }
}

// ------------------------------------------------------------------ canonical labels

__global__ void k_head(const i32 *__restrict__ comp, const i32 *__restrict__ minm, i64 n,
                       uint8_t *__restrict__ head)
{
    NODE_LOOP(n) head[u_] = minm[comp[u_]] == (i32)u_;
}

__global__ void k_label(const i32 *__restrict__ comp, const i32 *__restrict__ minm,
                        const i64 *__restrict__ rank, i64 n, i32 *__restrict__ lab)
{
    NODE_LOOP(n) lab[u_] = (i32)rank[minm[comp[u_]]];
}

// ------------------------------------------------------------------ forest
__global__ void k_forest_init(const i32 *__restrict__ a, const uint8_t *__restrict__ cyc,
                              const i32 *__restrict__ comp, const uint8_t *__restrict__ act,
                              i64 n, i32 *__restrict__ J0, i32 *__restrict__ D)
{
    NODE_LOOP(n)
    {
        i32 u = (i32)u_;
        if (!act[comp[u]]) continue;
        bool root = cyc[u] != 0;
        J0[u] = root ? u : a[u];
        D[u] = root ? 0 : 1;
    }
}

__global__ void k_forest_step(const i32 *__restrict__ comp, const uint8_t *__restrict__ act,
                              i64 n, const i32 *__restrict__ Jk, i32 *__restrict__ Jk1,
                              const i32 *__restrict__ Di, i32 *__restrict__ Do,
                              int *__restrict__ changed)
{
    NODE_LOOP(n)
    {
        i32 u = (i32)u_;
        if (!act[comp[u]]) continue;
        i32 x = Jk[u];
        i32 y = Jk[x];
        Jk1[u] = y;
        Do[u] = Di[u] + Di[x];
        if (y != x) *changed = 1;
    }
}

// Subtree sums: S_out = S_in, then S_out[J_k(u)] += S_in[u] for depth >= 2^k.
__global__ void k_sub_init(const i32 *__restrict__ comp, const uint8_t *__restrict__ act,
                           i64 n, const i32 *__restrict__ v32, const i64 *__restrict__ v64,
                           i64 *__restrict__ S)
{
    NODE_LOOP(n)
    {
        if (!act[comp[u_]]) continue;
        S[u_] = v32 ? (i64)v32[u_] : v64[u_];
    }
}

__global__ void k_sub_copy(const i32 *__restrict__ comp, const uint8_t *__restrict__ act,
                           i64 n, const i64 *__restrict__ Si, i64 *__restrict__ So)
{
    NODE_LOOP(n)
    {
        if (!act[comp[u_]]) continue;
        So[u_] = Si[u_];
    }
}

__global__ void k_sub_scatter(const i32 *__restrict__ comp, const uint8_t *__restrict__ act,
                              i64 n, const i32 *__restrict__ Jk, const i32 *__restrict__ depth,
                              int step, const i64 *__restrict__ Si, i64 *__restrict__ So)
{
    NODE_LOOP(n)
    {
        i32 u = (i32)u_;
        if (!act[comp[u]]) continue;
        if (depth[u] >= (1 << step)) {
            i64 v = Si[u];
            if (v) atomicAdd((unsigned long long *)&So[Jk[u]], (unsigned long long)v);
        }
    }
}

// The same for two value arrays at once (subtree strengths and cut
// corrections share the forest's loads): Sa from va32, Sb from vb64.
__global__ void k_sub_init2(const i32 *__restrict__ comp, const uint8_t *__restrict__ act, i64 n,
                            const i32 *__restrict__ va32, const i64 *__restrict__ vb64,
                            i64 *__restrict__ Sa, i64 *__restrict__ Sb)
{
    NODE_LOOP(n)
    {
        if (!act[comp[u_]]) continue;
        Sa[u_] = va32[u_];
        Sb[u_] = vb64[u_];
    }
}

__global__ void k_sub_copy2(const i32 *__restrict__ comp, const uint8_t *__restrict__ act, i64 n,
                            const i64 *__restrict__ Sai, const i64 *__restrict__ Sbi,
                            i64 *__restrict__ Sao, i64 *__restrict__ Sbo)
{
    NODE_LOOP(n)
    {
        if (!act[comp[u_]]) continue;
        Sao[u_] = Sai[u_];
        Sbo[u_] = Sbi[u_];
    }
}

__global__ void k_sub_scatter2(const i32 *__restrict__ comp, const uint8_t *__restrict__ act,
                               i64 n, const i32 *__restrict__ Jk, const i32 *__restrict__ depth,
                               int step, const i64 *__restrict__ Sai, const i64 *__restrict__ Sbi,
                               i64 *__restrict__ Sao, i64 *__restrict__ Sbo)
{
    NODE_LOOP(n)
    {
        i32 u = (i32)u_;
        if (!act[comp[u]]) continue;
        if (depth[u] >= (1 << step)) {
            const i32 x = Jk[u];
            const i64 va = Sai[u], vb = Sbi[u];
            if (va) atomicAdd((unsigned long long *)&Sao[x], (unsigned long long)va);
            if (vb) atomicAdd((unsigned long long *)&Sbo[x], (unsigned long long)vb);
        }
    }
}

__device__ __forceinline__ i32 lift(i32 u, int d, const i32 *J, i64 n)
{
    for (int k = 0; d; k++, d >>= 1)
        if (d & 1) u = J[(i64)k * n + u];
    return u;
}

// Lowest common ancestor of u (depth du) and v in one tree.  Most pairs meet
// within a few levels, so the deeper node climbs and both then climb
// together by parents (J_0) for up to LCA_WALK steps each; only pairs further
// apart take the jump tables.
#define LCA_WALK 8
__device__ __forceinline__ i32 lca(i32 u, int du, i32 v, const i32 *__restrict__ depth,
                                   const i32 *__restrict__ J, i64 n, int K)
{
    int dv = depth[v];
    if (du < dv) {
        i32 t = u;
        u = v;
        v = t;
        int s = du;
        du = dv;
        dv = s;
    }
    const int dd = du - dv;
    if (dd <= LCA_WALK) {
        for (int i = 0; i < dd; i++) u = J[u];
    } else {
        u = lift(u, dd, J, n);
    }
    if (u == v) return u;
    for (int st = 0; st < LCA_WALK; st++) {
        u = J[u];
        v = J[v];
        if (u == v) return u;
    }
    for (int k = K; k >= 0; k--) {
        i32 pu = J[(i64)k * n + u], pv = J[(i64)k * n + v];
        if (pu != pv) {
            u = pu;
            v = pv;
        }
    }
    return J[u];
}

// Row visitors: an operation on the entries of the rows whose community is
// in play.  begin() reads a row's state and says whether the row takes part
// (once per row, so rows of communities out of play cost one check), visit()
// handles one of its entries.  Rows run by degree bin from their descriptors
// (G lanes per row), hub rows by their chunks.
template <int G, class Op>
__global__ __launch_bounds__(G <= 64 ? SLM_BS : G) void k_visit_rows(LevelView L,
                                                                    const int4 *__restrict__ rowd,
                                                                    i64 count, Op op)
{
    constexpr int NG = G <= 64 ? SLM_BS / G : 1;
    const int gl = threadIdx.x % G;
    const i64 slot = (i64)blockIdx.x * NG + threadIdx.x / G;
    if (slot >= count) return;
    const int4 rd = rowd[slot];
    typename Op::Row R;
    if (!op.begin(rd.x, R)) return;
    const i64 e0 = (i64)(u32)rd.z | ((i64)rd.w << 32);
    for (int j = gl; j < rd.y; j += G) op.visit(R, L.e[e0 + j]);
}

template <class Op>
__global__ __launch_bounds__(SLM_BS) void k_visit_hub(LevelView L,
                                                     const HubChunk *__restrict__ hchunk, Op op)
{
    const HubChunk c = hchunk[blockIdx.x];
    typename Op::Row R;
    if (!op.begin(c.node, R)) return;
    for (i64 j = c.beg + threadIdx.x; j < c.end; j += SLM_BS) op.visit(R, L.e[j]);
}

template <class Op>
static void visit_rows(const LevelView &L, const Bins &Bn, const Op &op, hipStream_t s)
{
#define VISIT_BIN(B, G)                                                                \
    {                                                                                  \
        const i64 cnt = Bn.off[B + 1] - Bn.off[B];                                     \
        if (cnt > 0)                                                                   \
            k_visit_rows<G, Op><<<grid_for(cnt, G <= 64 ? SLM_BS / G : 1),               \
                                  G <= 64 ? SLM_BS : G, 0, s>>>(L, Bn.rowd + Bn.off[B], cnt, op); \
    }
    VISIT_BIN(BIN_8, 4)
    VISIT_BIN(BIN_32, 8)
    VISIT_BIN(BIN_64, 16)
    VISIT_BIN(BIN_128, 32)
    VISIT_BIN(BIN_256, 64)
    VISIT_BIN(BIN_512, 64)
    VISIT_BIN(BIN_1024, 128)
    VISIT_BIN(BIN_2048, 256)
    VISIT_BIN(BIN_4096, 512)
#undef VISIT_BIN
    if (Bn.nhub > 0) k_visit_hub<Op><<<(unsigned)Bn.nchunk, SLM_BS, 0, s>>>(L, Bn.hchunk, op);
}

// val[lca(u,v)] -= A_uv for every ordered pair (u,v), u != v, of one tree of
// an active community whose common ancestor is not the tree's root.  The
// matrix is symmetric, so each unordered pair is taken once, from its
// smaller end, with twice its weight.
struct LcaVisit {
    const i32 *comp;
    const uint8_t *act;
    const i32 *root, *depth, *J;
    i64 n;
    int K;
    i64 *val;
    struct Row {
        i32 u, c, r, du;
    };
    __device__ bool begin(i32 u, Row &R) const
    {
        R.u = u;
        R.c = comp[u];
        if (!act[R.c]) return false;
        R.r = root[u];
        R.du = depth[u];
        return true;
    }
    __device__ void visit(const Row &R, int2 ed) const
    {
        const i32 v = ed.x;
        // pairs meeting at their tree's root (a cycle node) are left out: no
        // cut uses the root's value, since a cycle node's move takes its
        // whole community
        if (R.du == 0 || v <= R.u || comp[v] != R.c || root[v] != R.r) return;
        const i32 l = lca(R.u, R.du, v, depth, J, n, K);
        if (l == R.r) return;
        atomicAdd((unsigned long long *)&val[l], (unsigned long long)(-2 * (i64)ed.y));
    }
};

// ------------------------------------------------------------------ block-aggregated totals
// out[key[i]] (op)= val[i] for i < n, with an LDS hash per workgroup so that
// a community spread over many nodes costs one global atomic per workgroup.
#define AGG_BS 1024
#define AGG_ITEMS 4
#define AGG_SLOTS 8192
template <bool MIN>
__global__ __launch_bounds__(AGG_BS) void k_agg(const i32 *__restrict__ key,
                                               const i32 *__restrict__ val, i64 n,
                                               i32 *__restrict__ out)
{
    __shared__ i32 hk[AGG_SLOTS];
    __shared__ i32 hv[AGG_SLOTS];
    for (int i = threadIdx.x; i < AGG_SLOTS; i += AGG_BS) {
        hk[i] = -1;
        hv[i] = MIN ? INT32_MAX : 0;
    }
    __syncthreads();
    const i64 base = (i64)blockIdx.x * AGG_BS * AGG_ITEMS;
    for (int r = 0; r < AGG_ITEMS; r++) {
        const i64 i = base + (i64)r * AGG_BS + threadIdx.x;
        if (i >= n) continue;
        const i32 c = key[i];
        const i32 v = MIN ? (i32)i : val[i];
        if (!MIN && v == 0) continue;
        u32 h = hash_label(c) >> (32 - 13);
        for (int probe = 0; probe < AGG_SLOTS; probe++) {
            i32 old = atomicCAS(&hk[h], -1, c);
            if (old == -1 || old == c) {
                if (MIN) atomicMin(&hv[h], v);
                else atomicAdd(&hv[h], v);
                break;
            }
            h = (h + 1) & (AGG_SLOTS - 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < AGG_SLOTS; i += AGG_BS) {
        const i32 c = hk[i];
        if (c < 0) continue;
        if (MIN) atomicMin(&out[c], hv[i]);
        else atomicAdd(&out[c], hv[i]);
    }
}

static void agg_add(const i32 *key, const i32 *val, i64 n, i32 *out, hipStream_t s)
{
    if (n > 0)
        k_agg<false><<<grid_for(n, AGG_BS * AGG_ITEMS), AGG_BS, 0, s>>>(key, val, n, out);
}

static void agg_min_index(const i32 *key, i64 n, i32 *out, hipStream_t s)
{
    if (n > 0)
        k_agg<true><<<grid_for(n, AGG_BS * AGG_ITEMS), AGG_BS, 0, s>>>(key, nullptr, n, out);
}

// ------------------------------------------------------------------ POSITIVE set-up
// g(u) = M2*(wc - A_uu) - k*(S_c - k) (+ y*(Y_c - y), directed model) < 0
// flags community c; the first such node numbers it.
__global__ void k_pos_flag(const i32 *__restrict__ comp, const i32 *__restrict__ k,
                           const i32 *__restrict__ diag, const i32 *__restrict__ wc,
                           const i32 *__restrict__ sig, const i32 *__restrict__ m2n, i64 m2,
                           const i32 *__restrict__ y, const i32 *__restrict__ sigy,
                           const uint8_t *__restrict__ active, i64 n, i32 *__restrict__ fidx,
                           i32 *__restrict__ flist, i64 *__restrict__ counters)
{
    NODE_LOOP(n)
    {
        i32 c = comp[u_];
        if (active && !active[c]) continue;
        i64 ku = k[u_];
        const i64 m2u = m2n ? (i64)m2n[u_] : m2;
        i64 g = m2u * (i64)(wc[u_] - diag[u_]) - ku * ((i64)sig[c] - ku);
        if (y) g += (i64)y[u_] * ((i64)sigy[c] - (i64)y[u_]);
        if (g >= 0) continue;
        if (atomicCAS(&fidx[c], -1, -2) == -1) {
            i32 f = (i32)atomicAdd((unsigned long long *)&counters[0], 1ull);
            flist[f] = c;
            fidx[c] = f;
        }
    }
}

// Member and cycle-node counts of the flagged communities.
__global__ void k_pos_count(const i32 *__restrict__ comp, const uint8_t *__restrict__ cyc,
                            const i32 *__restrict__ fidx, i64 n, i32 *__restrict__ fcnt,
                            i32 *__restrict__ flen)
{
    NODE_LOOP(n)
    {
        i32 f = fidx[comp[u_]];
        if (f < 0) continue;
        atomicAdd(&fcnt[f], 1);
        if (cyc[u_]) atomicAdd(&flen[f], 1);
    }
}

__global__ void k_pos_sizes(const i32 *__restrict__ flen, i64 nflag, i64 *__restrict__ wsz,
                            i64 *__restrict__ nsz)
{
    i64 f = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nflag) return;
    i64 l = flen[f];
    wsz[f] = l >= 2 ? l * l : 0;
    nsz[f] = l >= 2 ? l : 0;
}

__global__ void k_pos_scatter(const i32 *__restrict__ comp, const i32 *__restrict__ fidx, i64 n,
                              const i64 *__restrict__ mem_off, i32 *__restrict__ fill,
                              i32 *__restrict__ mem)
{
    NODE_LOOP(n)
    {
        i32 f = fidx[comp[u_]];
        if (f < 0) continue;
        i32 t = atomicAdd(&fill[f], 1);
        mem[mem_off[f] + t] = (i32)u_;
    }
}

// ------------------------------------------------------------------ MAXIMAL tails

// act[c]: community c holds a non-cycle candidate (its forest is needed);
// hasc[c]: c holds any candidate; ccnt[c]: its cycle candidates.
__global__ void k_max_cand(const i32 *__restrict__ lab, const i32 *__restrict__ best_c,
                           const uint8_t *__restrict__ cyc, i64 n, uint8_t *__restrict__ act,
                           uint8_t *__restrict__ hasc, i32 *__restrict__ ccnt,
                           i64 *__restrict__ counters)
{
    __shared__ i64 red[32];
    i64 cnt = 0;
    NODE_LOOP(n)
    {
        i32 c = lab[u_];
        if (best_c[u_] == c) continue;
        hasc[c] = 1;
        if (cyc[u_]) atomicAdd(&ccnt[c], 1);
        else act[c] = 1;
        cnt++;
    }
    cnt = block_sum<i64>(cnt, red);
    if (threadIdx.x == 0 && cnt) atomicAdd((unsigned long long *)&counters[0], (unsigned long long)cnt);
}

__global__ void k_max_clist(const i32 *__restrict__ lab, const i32 *__restrict__ best_c,
                            const uint8_t *__restrict__ cyc, i64 n, const i64 *__restrict__ coff,
                            i32 *__restrict__ cfill, i32 *__restrict__ clist)
{
    NODE_LOOP(n)
    {
        i32 c = lab[u_];
        if (best_c[u_] == c || !cyc[u_]) continue;
        i32 t = atomicAdd(&cfill[c], 1);
        clist[coff[c] + t] = (i32)u_;
    }
}

// Nearest non-cycle candidate ancestor-or-self (first marked ancestor by
// doubling); -1 when none lies below the cycle.
__global__ void k_nca_init(const i32 *__restrict__ lab, const uint8_t *__restrict__ act,
                           const i32 *__restrict__ best_c, const uint8_t *__restrict__ cyc,
                           const i32 *__restrict__ P, i64 n, i32 *__restrict__ F)
{
    NODE_LOOP(n)
    {
        i32 u = (i32)u_;
        i32 c = lab[u];
        if (!act[c] || cyc[u]) {
            F[u] = -1;
            continue;
        }
        bool marked = best_c[u] != c;
        i32 p = P[u];
        F[u] = marked ? u : (cyc[p] ? -1 : p);
    }
}

__global__ void k_nca_step(const i32 *__restrict__ lab, const i32 *__restrict__ best_c, i64 n,
                           const i32 *__restrict__ Fi, i32 *__restrict__ Fo)
{
    NODE_LOOP(n)
    {
        i32 f = Fi[u_];
        if (f < 0 || best_c[f] != lab[f]) Fo[u_] = f;
        else Fo[u_] = Fi[f];
    }
}

// w(B, D) of every candidate: each cross entry (u, v), D = lab v, adds its
// weight to the candidates whose tail holds u and whose target is D.
// w(B, D) for the candidates of MAXIMAL: every entry (u, v) from a community
// holding candidates to another community D adds its weight to the nearest
// candidate ancestors of u that move to D, and to the community's cycle
// candidates that move to D.
struct CrossVisit {
    const i32 *lab;
    const uint8_t *hasc, *act;
    const i32 *nca, *P, *best_c;
    const i64 *coff;
    const i32 *clist;
    i32 *wbd;
    struct Row {
        i32 u, c;
        bool act;
    };
    __device__ bool begin(i32 u, Row &R) const
    {
        R.u = u;
        R.c = lab[u];
        if (!hasc[R.c]) return false;
        R.act = act[R.c] != 0;
        return true;
    }
    __device__ void visit(const Row &R, int2 ed) const
    {
        const i32 D = lab[ed.x];
        if (D == R.c) return;
        if (R.act) {
            i32 x = nca[R.u];
            // every step climbs strictly; the bound only guards the loop
            for (int guard = 0; x >= 0 && guard < (1 << 30); guard++) {
                if (best_c[x] == D) atomicAdd(&wbd[x], ed.y);
                x = nca[P[x]];
            }
        }
        for (i64 t = coff[R.c]; t < coff[R.c + 1]; t++) {
            const i32 z = clist[t];
            if (best_c[z] == D) atomicAdd(&wbd[z], ed.y);
        }
    }
};

__device__ __forceinline__ u32 accept_draw(u64 seed, int level, int round, i32 node)
{
    // SplitMix64 (Steele, Lea & Flood 2014): output number ctr+1 of the stream
    // seeded with `seed`, ctr = level:16 | round:16 | node:32; high half.
    u64 ctr = ((u64)(uint16_t)level << 48) | ((u64)(uint16_t)round << 32) | (u64)(u32)node;
    u64 z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (u32)(z >> 32);
}

// move(B: c -> D) > 0 decides validity; valid moves draw.  In a batch the
// key uses the node's own graph total, the draw its graph's seed, level and
// local node number, and gvalid[g] counts the valid moves of graph g.
__global__ void k_max_valid(LevelView L, const i32 *__restrict__ lab,
                            const i32 *__restrict__ best_c, const uint8_t *__restrict__ cyc,
                            const i32 *__restrict__ sig, const i64 *__restrict__ subk,
                            const i64 *__restrict__ suby,
                            const i64 *__restrict__ cut, const i32 *__restrict__ wbd, u64 seed,
                            int level, int round, u64 accept_p, uint8_t *__restrict__ accept,
                            i64 *__restrict__ counters, unsigned long long *__restrict__ gvalid)
{
    __shared__ i64 red[32];
    const i64 n = L.n;
    i64 nv = 0, na = 0;
    // every lane of a wavefront runs the same iterations (seg_add_sorted)
    for (i64 b = (i64)blockIdx.x * blockDim.x; b < n; b += (i64)gridDim.x * blockDim.x) {
        const i64 u = b + threadIdx.x;
        bool ok = false;
        i32 g = -1;
        if (u < n) {
            const i32 i = (i32)u;
            g = L.gid ? L.gid[i] : 0;
            const i32 c = lab[i], D = best_c[i];
            accept[i] = 0;
            if (D != c) {
                i64 sb, tb, cb;
                if (cyc[i]) {
                    sb = sig[c];
                    tb = comm_y(L, c);
                    cb = 0;
                } else {
                    sb = subk[i];
                    tb = L.y ? suby[i] : 0;
                    cb = cut[i];
                }
                const i64 mv = node_m2(L, i) * ((i64)wbd[i] - cb) -
                               sb * ((i64)sig[D] - (i64)sig[c] + sb) +
                               tb * (comm_y(L, D) - comm_y(L, c) + tb);
                if (mv > 0) {
                    ok = true;
                    nv++;
                    u64 sd = seed;
                    int lv = level;
                    i32 loc = i;
                    if (L.gid) {
                        sd = L.gseed[g];
                        lv = L.glev[g];
                        loc = (i32)(u - L.gbase[g]);
                    }
                    if ((u64)accept_draw(sd, lv, round, loc) < accept_p) {
                        accept[i] = 1;
                        na++;
                    }
                }
            }
        }
        if (gvalid) seg_add_sorted(gvalid, g, ok ? 1 : 0);
    }
    nv = block_sum<i64>(nv, red);
    na = block_sum<i64>(na, red);
    if (threadIdx.x == 0) {
        if (nv) atomicAdd((unsigned long long *)&counters[1], (unsigned long long)nv);
        if (na) atomicAdd((unsigned long long *)&counters[2], (unsigned long long)na);
    }
}

// ------------------------------------------------------------------ modularity / compose
__global__ void k_nq_parts(const i32 *__restrict__ wc, i64 n, const i32 *__restrict__ sig,
                           const i32 *__restrict__ sigy, i64 nc, i64 *__restrict__ acc)
{
    __shared__ i64 red[32];
    i64 a = 0, b = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n || i < nc;
         i += (i64)gridDim.x * blockDim.x) {
        if (i < n) a += wc[i];
        if (i < nc) {
            b += (i64)sig[i] * (i64)sig[i];
            if (sigy) b -= (i64)sigy[i] * (i64)sigy[i];
        }
    }
    a = block_sum<i64>(a, red);
    b = block_sum<i64>(b, red);
    if (threadIdx.x == 0) {
        atomicAdd((unsigned long long *)&acc[0], (unsigned long long)a);
        atomicAdd((unsigned long long *)&acc[1], (unsigned long long)b);
    }
}

__global__ void k_compose(i32 *__restrict__ composed, const i32 *__restrict__ lab, i64 n0)
{
    NODE_LOOP(n0) composed[u_] = lab[composed[u_]];
}

// ================================================================== host side
void read_scalars(Work &W, const i64 *dev, int n, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(W.h_scal, dev, sizeof(i64) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

static int read_changed(Work &W, hipStream_t s)
{
    HIPCHK(hipMemcpyAsync(W.h_scal, W.changed, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return *(int *)W.h_scal;
}

static int ceil_log2(i64 n)
{
    int k = 0;
    while (((i64)1 << k) < n) k++;
    return k;
}

i64 canonical_labels(Work &W, i64 n, hipStream_t s)
{
    const unsigned g = node_grid(n);
    launch_fill_i32(W.minm, INT32_MAX, n, s);
    agg_min_index(W.comp, n, W.minm, s);
    k_head<<<g, SLM_BS, 0, s>>>(W.comp, W.minm, n, W.head);
    launch_scan_u8(W.head, W.rank, n, W.scan_tmp, s);
    k_label<<<g, SLM_BS, 0, s>>>(W.comp, W.minm, W.rank, n, W.lab);
    read_scalars(W, W.rank + n, 1, s);
    return W.h_scal[0];
}

i64 components(Work &W, const i32 *a, i64 n, bool want_lab, hipStream_t s)
{
    if (n == 0) return 0;
    const unsigned g = node_grid(n);
    const int K = ceil_log2(n) + 1;
    int2 *I = (int2 *)W.S0, *I2 = (int2 *)W.S1;
    k_comp_init<<<g, SLM_BS, 0, s>>>(a, n, I);
    launch_fill_i32(W.stepf, 0, K, s);
    for (int k = 0; k < K; k++) {
        k_comp_step<<<g, SLM_BS, 0, s>>>(I, I2, n, k ? W.stepf + k - 1 : nullptr, W.stepf + k);
        int2 *t = I;
        I = I2;
        I2 = t;
    }
    launch_fill_u8(W.cyc, 0, n, s);
    k_comp_mark<<<g, SLM_BS, 0, s>>>(I, n, W.comp, W.cyc);
    if (!want_lab) return -1;
    return canonical_labels(W, n, s);
}

// Forest of the active communities: jump tables J_0..J_K, depth, root.
static Forest build_forest(Work &W, const i32 *a, const i32 *comp, const uint8_t *act, i64 n,
                           hipStream_t s)
{
    const unsigned g = node_grid(n);
    k_forest_init<<<g, SLM_BS, 0, s>>>(a, W.cyc, comp, act, n, W.J, W.D0);
    i32 *Di = W.D0, *Do = W.D1;
    int k = 0;
    while (true) {
        if (k + 1 >= W.kmax) throw SlmError{4, "assignment forest deeper than the jump tables"};
        HIPCHK(hipMemsetAsync(W.changed, 0, sizeof(int), s));
        k_forest_step<<<g, SLM_BS, 0, s>>>(comp, act, n, W.J + (i64)k * n, W.J + (i64)(k + 1) * n,
                                           Di, Do, W.changed);
        i32 *t = Di;
        Di = Do;
        Do = t;
        if (!read_changed(W, s)) break;
        k++;
    }
    // J_k now maps every node to its root and Di holds exact depths
    Forest F;
    F.K = k;
    F.depth = Di;
    F.root = W.J + (i64)k * n;
    return F;
}

// out = subtree sums of v over the forest (doubling scatter).
static void subtree_sums(Work &W, const i32 *comp, const uint8_t *act, i64 n, const Forest &F,
                         const i32 *v32, const i64 *v64, i64 *out, hipStream_t s)
{
    const unsigned g = node_grid(n);
    i64 *Si = W.S0, *So = W.S1;
    k_sub_init<<<g, SLM_BS, 0, s>>>(comp, act, n, v32, v64, Si);
    for (int k = 0; k <= F.K; k++) {
        k_sub_copy<<<g, SLM_BS, 0, s>>>(comp, act, n, Si, So);
        k_sub_scatter<<<g, SLM_BS, 0, s>>>(comp, act, n, W.J + (i64)k * n, F.depth, k, Si, So);
        i64 *t = Si;
        Si = So;
        So = t;
    }
    HIPCHK(hipMemcpyAsync(out, Si, sizeof(i64) * n, hipMemcpyDeviceToDevice, s));
}

// subk = subtree sums of the strengths k, and cut(T_x) = w(T_x, c \ T_x) for
// every node of the active communities: subtree sums of w(u, c \ u) minus,
// at every lowest common ancestor, the weight of the tree pairs meeting
// there.  Both sums run in the same doubling passes.
static void subtree_strengths_cuts(Work &W, const LevelView &Lv, const Bins &B, const i32 *comp,
                                   const uint8_t *act, const Forest &F, const i32 *w_other,
                                   i64 *subk, i64 *cut, hipStream_t s)
{
    const i64 n = Lv.n;
    const unsigned g = node_grid(n);
    i64 *val = W.key;  // temporary
    k_sub_init<<<g, SLM_BS, 0, s>>>(comp, act, n, w_other, nullptr, val);
    if (Lv.nnz > 0)
        visit_rows(Lv, B, LcaVisit{comp, act, F.root, F.depth, W.J, n, F.K, val}, s);
    i64 *Ai = W.S0, *Ao = W.S1, *Bi = W.bestkey, *Bo = W.cbest_key;
    k_sub_init2<<<g, SLM_BS, 0, s>>>(comp, act, n, Lv.k, val, Ai, Bi);
    for (int k = 0; k <= F.K; k++) {
        k_sub_copy2<<<g, SLM_BS, 0, s>>>(comp, act, n, Ai, Bi, Ao, Bo);
        k_sub_scatter2<<<g, SLM_BS, 0, s>>>(comp, act, n, W.J + (i64)k * n, F.depth, k, Ai, Bi,
                                            Ao, Bo);
        i64 *t = Ai;
        Ai = Ao;
        Ao = t;
        t = Bi;
        Bi = Bo;
        Bo = t;
    }
    HIPCHK(hipMemcpyAsync(subk, Ai, sizeof(i64) * n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(cut, Bi, sizeof(i64) * n, hipMemcpyDeviceToDevice, s));
}


// Nodes that an accepted move changes: the mover (it ends in its target's
// community) and its old parent (it stays in what is left of the old one).
__global__ void k_mark_moves(const uint8_t *__restrict__ accept, const i32 *__restrict__ a, i64 n,
                             uint8_t *__restrict__ moved)
{
    NODE_LOOP(n)
    {
        if (!accept[u_]) continue;
        moved[u_] = 1;
        moved[a[u_]] = 1;
    }
}

__global__ void k_mark_comms(const i32 *__restrict__ comp, const uint8_t *__restrict__ moved,
                             i64 n, uint8_t *__restrict__ pact)
{
    NODE_LOOP(n)
    {
        if (moved[u_]) pact[comp[u_]] = 1;
    }
}

void mark_changed_communities(Work &W, i64 n, hipStream_t s)
{
    if (n == 0) return;
    launch_fill_u8(W.pact, 0, n, s);
    k_mark_comms<<<node_grid(n), SLM_BS, 0, s>>>(W.comp, W.moved, n, W.pact);
}

// With `active` (per community id of W.comp), only those communities are
// checked for a node of negative local gain: the caller knows the others
// are unchanged since POSITIVE left all their gains non-negative.
i64 positive(Work &W, const LevelView &Lv, const Bins &B, i64 *nc_out, hipStream_t s,
             const uint8_t *active)
{
    const i64 n = Lv.n;
    if (n == 0) {
        *nc_out = 0;
        return 0;
    }
    const unsigned g = node_grid(n);
    // communities (ids = cycle minima) holding a node of negative local gain
    launch_fill_i32(W.sigma, 0, n, s);
    agg_add(W.comp, Lv.k, n, W.sigma, s);
    if (Lv.y) {
        launch_fill_i32(W.sigy, 0, n, s);
        agg_add(W.comp, Lv.y, n, W.sigy, s);
    }
    run_own_weight(Lv, B, W.comp, active, W.wc, s);
    launch_fill_i32(W.fidx, -1, n, s);
    launch_fill_i64(W.counters, 0, 8, s);
    k_pos_flag<<<g, SLM_BS, 0, s>>>(W.comp, Lv.k, Lv.diag, W.wc, W.sigma, Lv.m2n, Lv.m2, Lv.y,
                                    W.sigy, active, n, W.fidx, W.flist, W.counters);
    read_scalars(W, W.counters, 1, s);
    const i64 nflag = W.h_scal[0];
    i64 splits = 0;
    if (nflag > 0) {
        // members of every flagged community, contiguous
        launch_fill_i32(W.fcnt, 0, nflag, s);
        launch_fill_i32(W.flen, 0, nflag, s);
        k_pos_count<<<g, SLM_BS, 0, s>>>(W.comp, W.cyc, W.fidx, n, W.fcnt, W.flen);
        launch_scan_i32(W.fcnt, W.mem_off, nflag, W.scan_tmp, s);
        launch_fill_i32(W.fcnt, 0, nflag, s);
        k_pos_scatter<<<g, SLM_BS, 0, s>>>(W.comp, W.fidx, n, W.mem_off, W.fcnt, W.mem);
        k_pos_sizes<<<grid_for(nflag, SLM_BS), SLM_BS, 0, s>>>(W.flen, nflag, W.wsz, W.nsz);
        launch_scan_i64(W.wsz, W.woff_f, nflag, W.scan_tmp, s);
        launch_scan_i64(W.nsz, W.noff_f, nflag, W.scan_tmp, s);
        read_scalars(W, W.woff_f + nflag, 1, s);
        const i64 wtotal = W.h_scal[0];
        dm_grow(*W.dm, W.W, W.W_cap, wtotal, 1024);
        HIPCHK(hipMemcpyAsync(W.part, W.comp, sizeof(i32) * n, hipMemcpyDeviceToDevice, s));
        launch_fill_i64(W.counters, 0, 1, s);
        PosArgs A;
        A.G = Lv;
        A.a = W.a;
        A.cyc = W.cyc;
        A.flist = W.flist;
        A.mem_off = W.mem_off;
        A.mem = W.mem;
        A.tmp = W.ptmp;
        A.ord = W.pord;
        A.chl = W.pchl;
        A.dpre = W.pdp;
        A.lvl = W.plvl;
        A.stk = W.pstk;
        A.part = W.part;
        A.win = W.win;
        A.subk = W.psub;
        A.cut = W.pcut;
        A.dep = W.pdep;
        A.root = W.proot;
        A.chs = W.chs;
        A.chc = W.chc;
        A.cpos = W.pos;
        A.lcyc = W.flen;
        A.woff = W.woff_f;
        A.W = W.W;
        A.noff = W.noff_f;
        A.cn = W.cnode;
        A.splits = W.counters;
        HIPCHK(hipMemsetAsync(W.changed, 0, sizeof(int), s));
        A.err = W.changed;
        if (Lv.y) launch_positive_dir(A, nflag, s);
        else launch_positive_wg(A, nflag, s);
        read_scalars(W, W.counters, 1, s);
        splits = W.h_scal[0];
        HIPCHK(hipMemcpyAsync(W.h_scal + 8, W.changed, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const int perr = *(int *)(W.h_scal + 8);
        if (perr) throw SlmError{4, "POSITIVE loop bound tripped (code " + std::to_string(perr) + ")"};
        HIPCHK(hipMemcpyAsync(W.comp, W.part, sizeof(i32) * n, hipMemcpyDeviceToDevice, s));
    }
    *nc_out = canonical_labels(W, n, s);
    return splits;
}

void community_totals(Work &W, const LevelView &Lv, const i32 *lab, i64 nc, hipStream_t s)
{
    launch_fill_i32(W.sigma, 0, nc, s);
    agg_add(lab, Lv.k, Lv.n, W.sigma, s);
    if (Lv.y) {
        launch_fill_i32(W.sigy, 0, nc, s);
        agg_add(lab, Lv.y, Lv.n, W.sigy, s);
    }
}

i64 maximal_moves(Work &W, const LevelView &Lv, const Bins &B, i64 nc, u64 seed, int level,
                  int round, u64 accept_p, i64 *stats, hipStream_t s, bool timing,
                  hipEvent_t ev0, hipEvent_t ev1, float *sweep_ms, unsigned long long *gvalid)
{
    const i64 n = Lv.n;
    const unsigned g = node_grid(n);
    community_totals(W, Lv, W.lab, nc, s);
    if (timing) HIPCHK(hipEventRecord(ev0, s));
    run_sweep(Lv, B, W.lab, W.sigma, W.best_c, W.delta, W.w_own, W.hub_part, W.hub_poff,
              W.hub_cwin, W.hub_tkey, W.hub_tid, s,
              W.fan.use(Lv.nnz));
    if (timing) HIPCHK(hipEventRecord(ev1, s));
    // candidates
    launch_fill_u8(W.act, 0, nc, s);
    launch_fill_u8(W.hasc, 0, nc, s);
    launch_fill_i32(W.ccnt, 0, nc, s);
    launch_fill_i64(W.counters, 0, 8, s);
    k_max_cand<<<g, SLM_BS, 0, s>>>(W.lab, W.best_c, W.cyc, n, W.act, W.hasc, W.ccnt, W.counters);
    read_scalars(W, W.counters, 1, s);
    if (timing) HIPCHK(hipEventElapsedTime(sweep_ms, ev0, ev1));
    const i64 ncand = W.h_scal[0];
    stats[0] = ncand;
    stats[1] = stats[2] = 0;
    if (ncand == 0) return 0;
    launch_scan_i32(W.ccnt, W.coff, nc, W.scan_tmp, s);
    launch_fill_i32(W.cfill, 0, nc, s);
    k_max_clist<<<g, SLM_BS, 0, s>>>(W.lab, W.best_c, W.cyc, n, W.coff, W.cfill, W.clist);
    // forest of the communities with non-cycle candidates
    Forest F = build_forest(W, W.a, W.lab, W.act, n, s);
    if (Lv.y) subtree_sums(W, W.lab, W.act, n, F, Lv.y, nullptr, W.suby, s);
    subtree_strengths_cuts(W, Lv, B, W.lab, W.act, F, W.w_own, W.subk, W.cut, s);
    // nearest candidate ancestors
    k_nca_init<<<g, SLM_BS, 0, s>>>(W.lab, W.act, W.best_c, W.cyc, W.J, n, W.nca0);
    i32 *Fi = W.nca0, *Fo = W.nca1;
    for (int k = 0; k <= F.K; k++) {
        k_nca_step<<<g, SLM_BS, 0, s>>>(W.lab, W.best_c, n, Fi, Fo);
        i32 *t = Fi;
        Fi = Fo;
        Fo = t;
    }
    launch_fill_i32(W.wbd, 0, n, s);
    const i64 entries = Lv.nnz;
    if (entries > 0)
        visit_rows(Lv, B, CrossVisit{W.lab, W.hasc, W.act, Fi, W.J, W.best_c, W.coff, W.clist,
                                     W.wbd}, s);
    k_max_valid<<<g, SLM_BS, 0, s>>>(Lv, W.lab, W.best_c, W.cyc, W.sigma, W.subk, W.suby, W.cut,
                                     W.wbd,
                                     seed, level, round, accept_p, W.accept, W.counters,
                                     gvalid);
    read_scalars(W, W.counters, 3, s);
    stats[1] = W.h_scal[1];
    stats[2] = W.h_scal[2];
    if (stats[1] == 0) return 0;
    HIPCHK(hipMemsetAsync(W.changed + 2, 0, sizeof(int), s));
    // the nodes whose communities the moves change, before the pointers do
    launch_fill_u8(W.moved, 0, n, s);
    k_mark_moves<<<g, SLM_BS, 0, s>>>(W.accept, W.a, n, W.moved);
    run_repoint(Lv, B, W.lab, W.best_c, W.accept, W.a, W.hub_ckey, W.hub_cid, W.changed + 2, s);
    HIPCHK(hipMemcpyAsync(W.h_scal, W.changed + 2, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (*(int *)W.h_scal)
        throw SlmError{4, "re-pointing found no neighbour in an accepted node's target community"};
    return stats[1];
}

i64 modularity_num(Work &W, const LevelView &Lv, const Bins &B, const i32 *lab, i64 nc,
                   hipStream_t s)
{
    community_totals(W, Lv, lab, nc, s);
    run_own_weight(Lv, B, lab, nullptr, W.wc, s);
    launch_fill_i64(W.counters, 0, 2, s);
    i64 m = Lv.n > nc ? Lv.n : nc;
    k_nq_parts<<<node_grid(m), SLM_BS, 0, s>>>(W.wc, Lv.n, W.sigma, Lv.y ? W.sigy : nullptr, nc,
                                               W.counters);
    read_scalars(W, W.counters, 2, s);
    return Lv.m2 * W.h_scal[0] - W.h_scal[1];
}

// Per-graph parts of N_Q in a batch.  Nodes and labels of one graph are
// contiguous, so the keys of consecutive lanes are sorted (seg_add_sorted).
__global__ void k_nq_graph(const i32 *__restrict__ wc, const i32 *__restrict__ gid, i64 n,
                           const i32 *__restrict__ sig, i64 nc, const i64 *__restrict__ gcb,
                           int G, unsigned long long *__restrict__ accI,
                           unsigned long long *__restrict__ accS)
{
    const i64 m = n > nc ? n : nc;
    for (i64 b = (i64)blockIdx.x * blockDim.x; b < m; b += (i64)gridDim.x * blockDim.x) {
        const i64 u = b + threadIdx.x;
        seg_add_sorted(accI, u < n ? gid[u] : -1, u < n ? (i64)wc[u] : 0);
        i32 g = -1;
        i64 sq = 0;
        if (u < nc) {
            int lo = 0, hi = G - 1;  // last g with gcb[g] <= u
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (gcb[mid] <= u) lo = mid;
                else hi = mid - 1;
            }
            g = lo;
            sq = (i64)sig[u] * (i64)sig[u];
        }
        seg_add_sorted(accS, g, sq);
    }
}

void modularity_graphs(Work &W, const LevelView &Lv, const Bins &B, const i32 *lab, i64 nc,
                       int G, const i64 *gcb, i64 *accI, i64 *accS, hipStream_t s)
{
    community_totals(W, Lv, lab, nc, s);
    run_own_weight(Lv, B, lab, nullptr, W.wc, s);
    launch_fill_i64(accI, 0, G, s);
    launch_fill_i64(accS, 0, G, s);
    const i64 m = Lv.n > nc ? Lv.n : nc;
    if (m > 0)
        k_nq_graph<<<node_grid(m), SLM_BS, 0, s>>>(W.wc, Lv.gid, Lv.n, W.sigma, nc, gcb, G,
                                                   (unsigned long long *)accI,
                                                   (unsigned long long *)accS);
}

void compose_labels(i32 *composed, const i32 *lab, i64 n0, hipStream_t s)
{
    if (n0 > 0) k_compose<<<node_grid(n0), SLM_BS, 0, s>>>(composed, lab, n0);
}
