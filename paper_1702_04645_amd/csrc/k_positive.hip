// POSITIVE (Sec. 3.3) with one workgroup per community that holds a node of
// negative local gain.  A community never interacts with another one during
// POSITIVE, so each workgroup runs the whole split sequence of its community
// (the while loop of the appendix POSITIVE) without leaving the kernel.
//
// The workgroup keeps, for every node u of the part P being split:
//   win(u)  = w(u, P \ u)                      -> g(u) = M2*win - k(S_P - k)
//   subk(u) = S over the subtree of u          (forest view: cycle nodes are
//   cut(u)  = w(T_u, P \ T_u)                   roots, parents are a(u))
// A branch cut at x (x non-cycle) removes T_x from P.  Instead of rebuilding
// P' = P \ T_x, the state is updated in place:
//   - S along the ancestors of x drops by subk(x);
//   - every entry (v, u) with v in T_x, u in P' lowers win(u) and win(v), the
//     cut of the nodes on the paths u -> lca and parent(x) -> lca (the pair
//     is no longer inside the part), and the cut of the nodes on v -> x
//     (inside T_x the pair now leaves the part);
//   - for a cycle of two or more nodes, the weight between the hanging trees.
// T_x keeps its subtree sums; its new root is x.  A cycle cut (self-assigning
// two cycle nodes) rebuilds both sides from scratch.  Keys:
//   branch x:      subk(x)(S_P - subk(x)) - M2 cut(x)
//   cycle (cp,cq): S_Y(S_P - S_Y) - M2 w(X, Y), Y = hanging trees at cycle
//                  positions p+1..q
// ties to the lowest (first, second) cut node; the best cut is applied even
// when its key is not positive, until no node of the part has g < 0.
//
// Split search.  A full scan of the part keeps, per lane, its PW_TOP best
// branch keys and its lowest gain as a candidate set; every other node is
// summarised by value buckets (by subtree strength for keys, by strength k
// for gains).  Between scans, a cut changes the key or gain of a node in two
// ways only: through S_P, which drops by D for everyone (a key falls by at
// least its bucket's floor times D, a gain rises by at least that much), and
// through the nodes whose own terms the cut updates (ancestors of x, nodes on
// the corrected cut paths, neighbours of T_x), which join the candidate set.
// The candidates are evaluated exactly at every split; when the bucket
// bounds cannot rule out a better key (ties included) or a negative gain
// outside the set, the part is scanned again.  The answer is therefore
// always the one a full scan would give.  T_x stays in the range (marked by
// its id) until the part is finished; it is then gathered from its root into
// a range of its own.
#include "slm_forest.h"

#define PW_BS 512
#define PW_NW (PW_BS / 64)

// Stack entries (s, e, part id, flags): ST_INIT rebuilds the part from its
// member range; ST_GATHER is a subtree cut off a part: its members are
// collected from its root when it is popped, into a range assigned when the
// part it left is finished (e holds its size until then, s = -1).
enum { ST_INIT = 1, ST_GATHER = 2 };

#define PW_CAND 4096  // candidate set of the split search
#define PW_TOP 4      // branch-key candidates kept per lane by a full scan
#define PW_NB 33      // value buckets: 0 for v <= 0, else 1 + floor(log2 v)
// membership of the candidate set: an open-addressing table of node ids in
// LDS, twice the set's size (a power of two), cleared at every full scan
#define PW_CT (2 * PW_CAND)
static_assert((PW_CT & (PW_CT - 1)) == 0, "the candidate table size must be a power of two");
constexpr int pw_ct_bits()
{
    int b = 0;
    while ((1 << b) < PW_CT) b++;
    return b;
}

struct PwShared {
    i64 red[2 * PW_NW + 2];
    int redf[PW_NW];
    i64 sig;       // S_P
    i64 bkey;      // best key
    u64 bpair;     // best (first, second)
    int neg;
    int sp;        // stack size
    int stop;      // the stack was empty at the last pop
    int s, e, pid, flags;
    int tail, head, lev_end;
    int L;         // cycle length of the part
    int chl_top;   // next free slot of the children arena
    int sp0;       // stack size when the current part started
    // split search: the nodes of the candidate set are evaluated exactly at
    // every split; every other node of the part is bounded by the bucket of
    // its value at the last full scan (see pw_bounds)
    int need_scan, ncand, cand_over, cand_cap;
    i64 sig_scan;  // S_P at the last full scan
    u64 kmax[PW_NB];  // per bucket of subtree strength: max branch key (order-mapped)
    u64 kpair[PW_NB]; // per bucket: lowest cut pair among its nodes whose key is that max
    u64 gmin[PW_NB];  // per bucket of strength: min local gain (order-mapped)
    i64 dpw[PW_BS + 1];  // degree-prefix window of one block of entries
    int snext;           // first member of the next block of entries
    i32 cand[PW_CAND];
    i32 ctab[PW_CT];     // node ids of the candidate set (-1: empty slot)
    short cslot[PW_CT];  // per table slot: the node's index in cand (-1: none)
    int cflag[PW_CAND];  // CF_DIRTY: cached terms stale; CF_GONE: left the part
};

enum { CF_DIRTY = 1, CF_GONE = 2 };

__device__ __forceinline__ u64 ord_map(i64 v) { return (u64)v ^ (1ull << 63); }
__device__ __forceinline__ i64 ord_unmap(u64 v) { return (i64)(v ^ (1ull << 63)); }
__device__ __forceinline__ int pw_bucket(i64 v) { return v <= 0 ? 0 : 64 - __clzll((u64)v); }
__device__ __forceinline__ i64 pw_floor(int b) { return b ? ((i64)1 << (b - 1)) : 0; }

// Bounds for the nodes outside the candidate set, from the value buckets of
// the last full scan; D = the drop of S_P since then.
//   thr: upper bound on their branch keys.  Such a node kept its subtree
//        strength and cut since the scan, so its key fell by (strength) * D;
//        a node of bucket b has strength >= pw_floor(b).  Only a node whose
//        key was its bucket's maximum can reach the bound, so tpair = the
//        lowest cut pair of those nodes over the buckets that reach it.
//   lb:  lower bound on their local gains g = M2 w_in - k (S_P - k), which
//        rose by k * D.
// One bucket per lane and a wavefront reduction; every lane of every
// wavefront gets the result.
__device__ __forceinline__ void pw_bounds(const PwShared &S, i64 D, i64 &thr, u64 &tpair,
                                          i64 &lb)
{
    const int lane = threadIdx.x & 63;
    i64 t = INT64_MIN, l = INT64_MAX;
    u64 tp = ~0ull;
    if (lane < PW_NB) {
        const u64 km = S.kmax[lane], gm = S.gmin[lane];
        if (km != 0) {
            t = ord_unmap(km) - pw_floor(lane) * D;
            tp = S.kpair[lane];
        }
        if (gm != ~0ull) l = ord_unmap(gm) + pw_floor(lane) * D;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const i64 ot = __shfl_xor(t, off, 64), ol = __shfl_xor(l, off, 64);
        const u64 otp = __shfl_xor(tp, off, 64);
        if (ot > t || (ot == t && otp < tp)) {
            t = ot;
            tp = otp;
        }
        l = min(l, ol);
    }
    thr = t;
    tpair = tp;
    lb = l;
}

__device__ __forceinline__ u32 pw_ct_hash(i32 v)
{
    return ((u32)v * 0x9E3779B1u) >> (32 - pw_ct_bits());
}

// Adds v to the candidate set once per scan; a node already in the set is
// marked dirty (its cached terms are re-read at the next evaluation).  Once
// the set has overflowed the next pass scans anyway, so nothing more is
// recorded; the table then holds at most PW_CAND + PW_BS ids.
__device__ __forceinline__ void pw_add_cand(PwShared &S, i32 v)
{
    if (S.cand_over) return;
    u32 h = pw_ct_hash(v);
    for (int probe = 0; probe < PW_CT; probe++, h = (h + 1) & (PW_CT - 1)) {
        const i32 old = atomicCAS(&S.ctab[h], -1, v);
        if (old == -1) {
            const int i = atomicAdd(&S.ncand, 1);
            if (i < S.cand_cap) {
                S.cand[i] = v;
                S.cflag[i] = CF_DIRTY;
                S.cslot[h] = (short)i;
            } else {
                S.cslot[h] = -1;
                S.cand_over = 1;
            }
            return;
        }
        if (old == v) {
            // the adder may not have stored the index yet: then a stale
            // index marks another candidate (a mark only forces a re-read),
            // and the adder's own flag is dirty anyway.  The mark is an
            // atomic OR: a plain read-modify-write could store a flag read
            // before a concurrent add reset that slot
            const int c = S.cslot[h];
            if (c >= 0 && c < S.cand_cap) atomicOr(&S.cflag[c], CF_DIRTY);
            return;
        }
    }
    S.cand_over = 1;  // table full (not reached: it has room for every add)
}

// A candidate that leaves the part with a cut-off subtree.  Adds of other
// nodes may run concurrently (the entry pass of a one-node cut); v itself is
// never being added then, and its slot and index were settled by an earlier
// barrier, so a probe either finds them or ends at an empty slot.
__device__ __forceinline__ void pw_drop_cand(PwShared &S, i32 v)
{
    u32 h = pw_ct_hash(v);
    for (int probe = 0; probe < PW_CT; probe++, h = (h + 1) & (PW_CT - 1)) {
        const i32 k = S.ctab[h];
        if (k == -1) return;
        if (k == v) {
            const int c = S.cslot[h];
            if (c >= 0 && c < S.cand_cap && S.cand[c] == v) atomicOr(&S.cflag[c], CF_GONE);
            return;
        }
    }
}

// Ranges for the subtrees cut off the finished part: consecutive from off.
__device__ __forceinline__ void pw_assign(int4 *STK, int from, int to, int off)
{
    for (int k = from; k < to; k++) {
        int4 t = STK[k];
        if ((t.w & ST_GATHER) && t.x < 0) {
            const int sz = t.y;
            t.x = off;
            t.y = off + sz;
            off += sz;
            STK[k] = t;
        }
    }
}

__device__ __forceinline__ i64 wg_sum(i64 v, PwShared &S)
{
    v = group_sum<64>(v);
    const int wid = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) S.red[wid] = v;
    __syncthreads();
    i64 t = 0;
    for (int w = 0; w < PW_NW; w++) t += S.red[w];
    __syncthreads();
    return t;
}

// Best (key desc, pair asc) over the workgroup plus the OR of one flag per
// thread, with one barrier.  It relies on its caller for the other two: every
// earlier reader of S.red has passed a barrier since (the other reductions end
// with one, and the split loop passes one between two calls), and no thread
// writes S.red again before the next barrier.
__device__ __forceinline__ void wg_best_or(i64 &key, u64 &pair, int &flag, PwShared &S)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        i64 ok = __shfl_xor(key, off, 64);
        u64 op = __shfl_xor(pair, off, 64);
        flag |= __shfl_xor(flag, off, 64);
        if (ok > key || (ok == key && op < pair)) {
            key = ok;
            pair = op;
        }
    }
    const int wid = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        S.red[2 * wid] = key;
        S.red[2 * wid + 1] = (i64)pair;
        S.redf[wid] = flag;
    }
    __syncthreads();
    key = S.red[0];
    pair = (u64)S.red[1];
    flag = S.redf[0];
    for (int w = 1; w < PW_NW; w++) {
        i64 k2 = S.red[2 * w];
        u64 p2 = (u64)S.red[2 * w + 1];
        flag |= S.redf[w];
        if (k2 > key || (k2 == key && p2 < pair)) {
            key = k2;
            pair = p2;
        }
    }
}

// Exclusive scan of one value per thread over the workgroup; *total = sum.
__device__ __forceinline__ i64 wg_scan(i64 v, i64 &total, PwShared &S)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
    i64 inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        i64 t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    __syncthreads();
    if (lane == 63) S.red[wid] = inc;
    __syncthreads();
    i64 before = 0, tot = 0;
    for (int w = 0; w < PW_NW; w++) {
        if (w < wid) before += S.red[w];
        tot += S.red[w];
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

// Adds val into dst[idx] with one atomic per run of equal idx inside the
// wave.  idx must be non-decreasing over the in-range lanes of the wave, so
// equal keys form one run; lanes out of range pass in_range = false, lanes
// filtered out keep their key and pass val = 0.
__device__ __forceinline__ void wave_run_add(bool in_range, i32 idx, i64 val, i32 *dst)
{
    const int lane = threadIdx.x & 63;
    i32 key = in_range ? idx : -1;
    i64 v = in_range ? val : 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        i64 t = __shfl_up(v, d, 64);
        i32 k2 = __shfl_up(key, d, 64);
        if (lane >= d && k2 == key) v += t;
    }
    i32 nxt = __shfl_down(key, 1, 64);
    bool last = (lane == 63) || nxt != key;
    if (in_range && last && v != 0) atomicAdd(&dst[idx], (i32)v);
}

// Every loop of the kernel is bounded by the part size; a bound that trips
// (which a consistent state never does) records an error code and ends the
// workgroup's work instead of spinning.
__device__ __forceinline__ void report(int *err, int code)
{
    atomicCAS(err, 0, code);
}

// Flattened walk over the CSR entries of nodes list[0..cnt): degree prefix
// into dp[0..cnt], then entry t of the list belongs to list[upper(dp, t)-1].
__device__ __forceinline__ i64 wg_degree_prefix(const i32 *list, int cnt, const i64 *rp, i64 *dp,
                                                PwShared &S)
{
    i64 carry = 0;
    for (int b = 0; b < cnt; b += PW_BS) {
        int i = b + threadIdx.x;
        i64 d = i < cnt ? rp[list[i] + 1] - rp[list[i]] : 0;
        i64 tot;
        i64 ex = wg_scan(d, tot, S);
        if (i < cnt) dp[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) dp[cnt] = carry;
    __syncthreads();
    return carry;
}

__device__ __forceinline__ int find_slot(const i64 *dp, int cnt, i64 t)
{
    int lo = 0, hi = cnt;  // dp[lo] <= t < dp[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (dp[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Member (slot, with its prefix dp[slot]) of entry t = b + threadIdx.x of a
// flattened member list with prefix dp[0..cnt], for the block [b, b+PW_BS)
// whose first entry belongs to member s_lo.  The block's prefix values are
// staged in LDS: every member of a community has an entry, so a block spans
// at most PW_BS + 1 of them (a member beyond that window is searched in dp
// itself).  *s_next gets the member of the block's last entry, the first
// member of the next block.  Every thread of the workgroup calls it.
__device__ __forceinline__ void wg_block_slot(const i64 *dp, int cnt, i64 tot, i64 b, int s_lo,
                                              int &slot, i64 &d0, int &s_next, PwShared &S)
{
    const int j = s_lo + threadIdx.x;
    S.dpw[threadIdx.x] = j <= cnt ? dp[j] : INT64_MAX;
    if (threadIdx.x == 0) S.dpw[PW_BS] = s_lo + PW_BS <= cnt ? dp[s_lo + PW_BS] : INT64_MAX;
    __syncthreads();
    const i64 t = b + threadIdx.x;
    slot = 0;
    d0 = 0;
    if (t < tot) {
        if (S.dpw[PW_BS] <= t) {
            slot = find_slot(dp, cnt, t);
            d0 = dp[slot];
        } else {
            int lo = 0, hi = PW_BS;  // dpw[lo] <= t < dpw[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (S.dpw[mid] <= t) lo = mid;
                else hi = mid;
            }
            slot = s_lo + lo;
            d0 = S.dpw[lo];
        }
    }
    if (threadIdx.x == PW_BS - 1) S.snext = slot;
    __syncthreads();
    s_next = S.snext;
}

// Stable partition of r[0..m): members with keep(u) first; others after.
// Uses out as temporary; returns the number kept.
template <class Keep>
__device__ int wg_partition(i32 *r, int m, i32 *out, Keep keep, PwShared &S)
{
    i64 carry_k = 0, carry_o = 0;
    // count kept first
    i64 nk = 0;
    for (int b = 0; b < m; b += PW_BS) {
        int i = b + threadIdx.x;
        nk += (i < m && keep(r[i])) ? 1 : 0;
    }
    nk = wg_sum(nk, S);
    for (int b = 0; b < m; b += PW_BS) {
        int i = b + threadIdx.x;
        bool ok = i < m;
        i32 u = ok ? r[i] : 0;
        bool k = ok && keep(u);
        i64 tk, to;
        i64 ek = wg_scan(k ? 1 : 0, tk, S);
        i64 eo = wg_scan((ok && !k) ? 1 : 0, to, S);
        if (k) out[carry_k + ek] = u;
        else if (ok) out[nk + carry_o + eo] = u;
        carry_k += tk;
        carry_o += to;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += PW_BS) r[i] = out[i];
    __syncthreads();
    return (int)nk;
}

__global__ __launch_bounds__(PW_BS) void k_positive_wg(PosArgs A)
{
    __shared__ PwShared S;
    const int f = blockIdx.x;
    const i64 base = A.mem_off[f];
    const int m0 = (int)(A.mem_off[f + 1] - base);
    i32 *M = A.mem + base;
    i32 *TMP = A.tmp + base;
    i32 *ORD = A.ord + base;
    i32 *CHL = A.chl + 2 * base;  // arena of 2*m0 slots: every part built from
                                  // scratch takes fresh slots, so the children
                                  // lists of parts waiting on the stack survive
    i64 *DP = A.dpre + base + f;
    int4 *STK = A.stk + base;
    const int Lc0 = A.lcyc[f];
    i64 *Wm = Lc0 >= 2 ? A.W + A.woff[f] : nullptr;  // (L x L) weights between hanging trees
    i32 *CN = A.cn + A.noff[f];
    const LevelView &G = A.G;
    const i64 m2 = node_m2(G, M[0]);  // every member belongs to one graph
    i32 *a = A.a;
    uint8_t *cyc = A.cyc;

    // candidate cache in LDS (the kernel's registers allow one workgroup per
    // CU, so its LDS is there): at most min(PW_CAND, m0) entries
    __shared__ int4 CV[PW_CAND];
    // iterations: at most one pass per part and, per split, one full scan
    // and one split step; parts and splits are fewer than 2*m0
    const int iter_cap = 6 * m0 + 16;

    if (threadIdx.x == 0) {
        STK[0] = make_int4(0, m0, A.flist[f], ST_INIT);
        S.sp = 1;
        S.chl_top = 0;
        S.cand_cap = m0 < PW_CAND ? m0 : PW_CAND;
    }
    __syncthreads();
    int iters = 0;  // every thread counts the same passes (uniform loops)
    while (true) {
        // thread 0 pops the next part, or records that the stack is empty,
        // between two barriers; every thread decides from that record, never
        // from the stack size, which the pop changes
        __syncthreads();
        if (threadIdx.x == 0) {
            S.stop = S.sp == 0;
            if (!S.stop) {
                int4 t = STK[--S.sp];
                S.s = t.x;
                S.e = t.y;
                S.pid = t.z;
                S.flags = t.w;
                S.sp0 = S.sp;
                S.need_scan = 1;
            }
        }
        __syncthreads();
        if (S.stop) break;
        if (++iters > iter_cap) {
            if (threadIdx.x == 0) report(A.err, 5);
            break;
        }
        if (S.s < 0 || S.e < S.s || S.e > m0) {  // a range outside the community
            if (threadIdx.x == 0) report(A.err, 9);
            break;
        }
        const int s = S.s, pid = S.pid;
        if (S.e - s <= 1) continue;
        // -------------------------------------------------- (re)build a part
        if (S.flags & ST_INIT) {
            const int m = S.e - s;
            i32 *P = M + s;
            i64 sg = 0, nl = 0;
            for (int i = threadIdx.x; i < m; i += PW_BS) {
                i32 u = P[i];
                A.part[u] = pid;
                A.win[u] = 0;
                A.chc[u] = 0;
                A.subk[u] = G.k[u];
                sg += G.k[u];
                nl += cyc[u] ? 1 : 0;
            }
            sg = wg_sum(sg, S);
            nl = wg_sum(nl, S);
            if (threadIdx.x == 0) {
                S.sig = sg;
                S.L = (int)nl;
            }
            // children lists (contiguous per parent), positions absolute in CHL
            for (int i = threadIdx.x; i < m; i += PW_BS) {
                i32 u = P[i];
                if (!cyc[u]) atomicAdd(&A.chc[a[u]], 1);
            }
            __syncthreads();
            {
                const int arena = S.chl_top;
                i64 carry = 0;
                for (int b = 0; b < m; b += PW_BS) {
                    int i = b + threadIdx.x;
                    i64 c = i < m ? A.chc[P[i]] : 0;
                    i64 tot;
                    i64 ex = wg_scan(c, tot, S);
                    if (i < m) A.chs[P[i]] = (i32)(arena + carry + ex);
                    carry += tot;
                }
                __syncthreads();
                if (threadIdx.x == 0) S.chl_top = arena + m;
            }
            for (int i = threadIdx.x; i < m; i += PW_BS) A.chc[P[i]] = 0;
            __syncthreads();
            for (int i = threadIdx.x; i < m; i += PW_BS) {
                i32 u = P[i];
                if (!cyc[u]) {
                    i32 p = a[u];
                    int slot = atomicAdd(&A.chc[p], 1);
                    CHL[A.chs[p] + slot] = u;
                }
            }
            __syncthreads();
            // level order from the cycle nodes (children of a node stay contiguous)
            if (threadIdx.x == 0) S.tail = 0;
            __syncthreads();
            for (int i = threadIdx.x; i < m; i += PW_BS) {
                i32 u = P[i];
                if (cyc[u]) {
                    int q = atomicAdd(&S.tail, 1);
                    ORD[q] = u;
                    A.dep[u] = 0;
                    A.root[u] = u;
                }
            }
            __syncthreads();
            // cycle positions along a, from the smallest cycle node
            if (S.L >= 2 && threadIdx.x == 0) {
                i32 z = INT32_MAX;
                for (int q = 0; q < S.L; q++) z = min(z, ORD[q]);
                i32 y = z;
                for (int j = 0; j < S.L; j++) {
                    CN[j] = y;
                    A.cpos[y] = j;
                    y = a[y];
                }
            }
            int lev_b = 0;
            if (threadIdx.x == 0) {
                S.head = 0;
                S.lev_end = S.tail;
            }
            __syncthreads();
            int nlev = 0;
            while (true) {
                const int lb = S.head, le = S.lev_end;
                if (lb == le) break;
                if (threadIdx.x == 0) A.lvl[base + f + nlev] = lb;
                nlev++;
                for (int i = lb + threadIdx.x; i < le; i += PW_BS) {
                    i32 u = ORD[i];
                    int c = A.chc[u];
                    if (c) {
                        int q = atomicAdd(&S.tail, c);
                        int cs = A.chs[u];
                        for (int j = 0; j < c; j++) {
                            i32 ch = CHL[cs + j];
                            ORD[q + j] = ch;
                            A.dep[ch] = A.dep[u] + 1;
                            A.root[ch] = A.root[u];
                        }
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    S.head = le;
                    S.lev_end = S.tail;
                }
                __syncthreads();
            }
            if (threadIdx.x == 0) A.lvl[base + f + nlev] = m;
            (void)lev_b;
            // win, and the intra-part entries between different hanging trees
            const int L = S.L;
            if (L >= 2)
                for (int i = threadIdx.x; i < L * L; i += PW_BS) Wm[i] = 0;
            const i64 tot = wg_degree_prefix(P, m, G.rp, DP, S);
            for (i64 b = 0, sl = 0; b < tot; b += PW_BS) {
                const i64 t = b + threadIdx.x;
                int slot, snx;
                i64 d0;
                wg_block_slot(DP, m, tot, b, (int)sl, slot, d0, snx, S);
                sl = snx;
                i32 u = 0;
                i64 val = 0;
                if (t < tot) {
                    u = P[slot];
                    int2 ed = G.e[G.rp[u] + (t - d0)];
                    i32 v = ed.x;
                    if (v != u && A.part[v] == pid) {
                        val = ed.y;
                        if (L >= 2 && A.root[u] != A.root[v])
                            atomicAdd((unsigned long long *)&Wm[A.cpos[A.root[u]] * L +
                                                                 A.cpos[A.root[v]]],
                                      (unsigned long long)(i64)ed.y);
                    }
                }
                wave_run_add(t < tot, u, val, A.win);
            }
            __syncthreads();
            // cut(u) = subtree sum of win minus, at every lowest common ancestor
            // inside one tree, the weight of the pairs meeting there
            for (int i = threadIdx.x; i < m; i += PW_BS) A.cut[P[i]] = A.win[P[i]];
            __syncthreads();
            for (i64 b = 0, sl = 0; b < tot; b += PW_BS) {
                const i64 t = b + threadIdx.x;
                int slot, snx;
                i64 d0;
                wg_block_slot(DP, m, tot, b, (int)sl, slot, d0, snx, S);
                sl = snx;
                if (t < tot) {
                    i32 u = P[slot];
                    int2 ed = G.e[G.rp[u] + (t - d0)];
                    i32 v = ed.x;
                    // the matrix is symmetric: each pair once, from its
                    // smaller end, with both directions' weight
                    if (v > u && A.part[v] == pid && A.root[u] == A.root[v] && A.dep[u] != 0 &&
                        A.dep[v] != 0) {
                        // (a pair with the root meets at a cycle node, which
                        // takes no correction)
                        i32 x = u, y = v;
                        int dx = A.dep[u], dy = A.dep[v];
                        int guard = 0;
                        // inside a tree a parent is one level up, so the
                        // depths are counted down; a walk takes at most
                        // 2 (m - 1) steps
                        while (dx > dy && guard++ < 2 * m) {
                            x = a[x];
                            dx--;
                        }
                        while (dy > dx && guard++ < 2 * m) {
                            y = a[y];
                            dy--;
                        }
                        while (x != y && guard++ < 2 * m) {
                            x = a[x];
                            y = a[y];
                        }
                        if (guard >= 2 * m) report(A.err, 1);
                        else if (!cyc[x]) atomicSub(&A.cut[x], 2 * ed.y);
                    }
                }
            }
            __syncthreads();
            // subtree sums, deepest level first (siblings are contiguous)
            for (int l = nlev - 1; l >= 1; l--) {
                const int lb = A.lvl[base + f + l], le = A.lvl[base + f + l + 1];
                for (int b = lb; b < le; b += PW_BS) {
                    const int i = b + threadIdx.x;
                    bool on = i < le;
                    i32 u = on ? ORD[i] : 0;
                    i32 p = on ? a[u] : 0;
                    bool toroot = on && cyc[p];
                    wave_run_add(on, p, (on && (L >= 2 || !toroot)) ? A.subk[u] : 0, A.subk);
                    wave_run_add(on, p, (on && !toroot) ? A.cut[u] : 0, A.cut);
                }
                __syncthreads();
            }
        } else {
            // ST_GATHER: T_x, cut off an earlier part, is the subtree of its
            // root x over the children lists, restricted to the nodes that
            // still carry its id; its range holds exactly its members.
            const int m = S.e - s;
            i32 *P = M + s;
            if (threadIdx.x == 0) {
                P[0] = pid;
                S.head = 0;
                S.tail = 1;
                S.lev_end = 1;
            }
            __syncthreads();
            for (int lv = 0; lv <= m; lv++) {
                const int lb = S.head, le = S.lev_end;
                if (lb == le) break;
                for (int i = lb + threadIdx.x; i < le; i += PW_BS) {
                    const i32 u = P[i];
                    const int c = A.chc[u], cs = A.chs[u];
                    for (int j = 0; j < c; j++) {
                        const i32 ch = CHL[cs + j];
                        if (A.part[ch] != pid) continue;
                        const int q = atomicAdd(&S.tail, 1);
                        if (q < m) P[q] = ch;
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    S.head = le;
                    S.lev_end = min(S.tail, m);
                }
                __syncthreads();
            }
            if (S.tail != m) {
                if (threadIdx.x == 0) report(A.err, 8);
                break;
            }
            i64 sg = 0;
            for (int i = threadIdx.x; i < m; i += PW_BS) sg += G.k[P[i]];
            sg = wg_sum(sg, S);
            // the first pass would scan the part and stop at once unless a
            // member has a negative local gain: decide that here
            i64 nneg = 0;
            for (int i = threadIdx.x; i < m; i += PW_BS) {
                const i32 u = P[i];
                const i64 ku = G.k[u];
                if (m2 * (i64)A.win[u] - ku * (sg - ku) < 0) nneg++;
            }
            nneg = wg_sum(nneg, S);
            if (threadIdx.x == 0) {
                S.sig = sg;
                S.L = 1;
            }
            __syncthreads();
            if (nneg == 0) continue;  // no split: the part is final
        }
        // -------------------------------------------------- split loop
        // every pass of this loop starts after a barrier (the part's set-up or
        // the end of the previous pass), so the shared state is settled
        while (true) {
            if (++iters > iter_cap) {
                if (threadIdx.x == 0) report(A.err, 6);
                break;
            }
            int m = S.e - s;
            i32 *P = M + s;
            const i64 sig = S.sig;
            const int L = S.L;
            if (m <= 1) break;
            const bool scanned = S.need_scan != 0 || S.cand_over != 0;
            i64 bk = INT64_MIN;
            u64 bp = ~0ull;
            int neg = 0;
            if (scanned) {
                // ---- full scan of the range; nodes that left the part are
                // skipped.  Every lane keeps its best branch key and its
                // lowest gain as candidates; all other nodes go to the
                // buckets that bound them until the next scan.
                for (int b = threadIdx.x; b < PW_NB; b += PW_BS) {
                    S.kmax[b] = 0;
                    S.kpair[b] = ~0ull;
                    S.gmin[b] = ~0ull;
                }
                for (int i = threadIdx.x; i < PW_CT; i += PW_BS) S.ctab[i] = -1;
                __syncthreads();  // every thread has read need_scan
                if (threadIdx.x == 0) {
                    S.ncand = 0;
                    S.cand_over = 0;
                    S.sig_scan = sig;
                    S.need_scan = 0;
                }
                __syncthreads();
                // per lane: the PW_TOP best (key desc, pair asc) branch keys,
                // sorted; a node pushed out goes to its bucket
                i64 tk[PW_TOP], ts[PW_TOP];
                u64 tp[PW_TOP];
#pragma unroll
                for (int q = 0; q < PW_TOP; q++) {
                    tk[q] = INT64_MIN;
                    tp[q] = ~0ull;
                    ts[q] = 0;
                }
                i32 gu = -1;
                i64 gm = INT64_MAX, gk = 0, live = 0;
                constexpr int SU = 8;
                for (int i0 = threadIdx.x; i0 < m; i0 += PW_BS * SU) {
                    i32 uu[SU], pp[SU], ww[SU], sxv[SU], cxv[SU], kk[SU];
                    uint8_t cy[SU];
#pragma unroll
                    for (int j = 0; j < SU; j++) {
                        const int i = i0 + j * PW_BS;
                        uu[j] = i < m ? P[i] : -1;
                    }
#pragma unroll
                    for (int j = 0; j < SU; j++) {
                        pp[j] = -1;
                        kk[j] = ww[j] = sxv[j] = cxv[j] = 0;
                        cy[j] = 1;
                        if (uu[j] >= 0) {
                            const i32 u = uu[j];
                            pp[j] = A.part[u];
                            kk[j] = G.k[u];
                            ww[j] = A.win[u];
                            cy[j] = cyc[u];
                            sxv[j] = A.subk[u];
                            cxv[j] = A.cut[u];
                        }
                    }
#pragma unroll
                    for (int j = 0; j < SU; j++) {
                        const int i = i0 + j * PW_BS;
                        if (uu[j] < 0) continue;
                        // the branch key and bucket of position i, for the
                        // pass below (INT64_MIN: no branch cut there)
                        DP[i] = INT64_MIN;
                        if (pp[j] != pid) continue;
                        const i32 u = uu[j];
                        live++;
                        const i64 ku = kk[j];
                        const i64 g = m2 * (i64)ww[j] - ku * (sig - ku);
                        if (g < gm) {
                            if (gu >= 0) atomicMin((unsigned long long *)&S.gmin[pw_bucket(gk)], (unsigned long long)ord_map(gm));
                            gm = g;
                            gu = u;
                            gk = ku;
                        } else {
                            atomicMin((unsigned long long *)&S.gmin[pw_bucket(ku)], (unsigned long long)ord_map(g));
                        }
                        if (!cy[j]) {
                            i64 ck = sxv[j] * (sig - sxv[j]) - m2 * (i64)cxv[j];
                            u64 cp = ((u64)(u32)u << 32) | (u64)(u32)u;
                            i64 cs = sxv[j];
                            DP[i] = ck;
                            TMP[i] = pw_bucket(cs);
                            // insert into the sorted top list; what falls off
                            // the end goes to its bucket
#pragma unroll
                            for (int q = 0; q < PW_TOP; q++) {
                                if (ck > tk[q] || (ck == tk[q] && cp < tp[q])) {
                                    const i64 k2 = tk[q], s2 = ts[q];
                                    const u64 p2 = tp[q];
                                    tk[q] = ck;
                                    tp[q] = cp;
                                    ts[q] = cs;
                                    ck = k2;
                                    cp = p2;
                                    cs = s2;
                                }
                            }
                            if (cp != ~0ull)
                                atomicMax((unsigned long long *)&S.kmax[pw_bucket(cs)], (unsigned long long)ord_map(ck));
                        }
                    }
                }
                bk = tk[0];
                bp = tp[0];
                neg = gm < 0 ? 1 : 0;
                __syncthreads();
                // lowest pair among the bucket nodes that hold their bucket's
                // maximum key (the lane bests are candidates, not bucket
                // nodes); the keys and buckets were kept by position, so this
                // pass reads three coalesced arrays (each position is read by
                // the thread that wrote it)
                for (int i = threadIdx.x; i < m; i += PW_BS) {
                    const i64 key = DP[i];
                    if (key == INT64_MIN) continue;
                    const i32 u = P[i];
                    const u64 pr = ((u64)(u32)u << 32) | (u64)(u32)u;
                    bool top = false;
#pragma unroll
                    for (int q = 0; q < PW_TOP; q++) top |= tp[q] == pr;
                    if (top) continue;
                    const int b = TMP[i];
                    if (ord_map(key) == S.kmax[b])
                        atomicMin((unsigned long long *)&S.kpair[b], (unsigned long long)pr);
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < PW_TOP; q++)
                    if (tp[q] != ~0ull) pw_add_cand(S, (i32)(tp[q] >> 32));
                if (gu >= 0) pw_add_cand(S, gu);
                live = wg_sum(live, S);
                if (m > 2 * live + PW_BS) {  // most of the range has left: compact
                    const int kept =
                        wg_partition(P, m, ORD, [&](i32 u) { return A.part[u] == pid; }, S);
                    if (threadIdx.x == 0) S.e = s + kept;
                    __syncthreads();
                    m = kept;
                }
            } else {
                // ---- the candidate set, exactly: clean candidates from the
                // cache (their terms are unchanged since read), dirty ones
                // from the node arrays
                const int nc = min(S.ncand, S.cand_cap);
                i64 gm = INT64_MAX;
                for (int i = threadIdx.x; i < nc; i += PW_BS) {
                    const int fl = S.cflag[i];
                    if (fl & CF_GONE) continue;
                    const i32 u = S.cand[i];
                    int4 cv;
                    if (fl & CF_DIRTY) {
                        // the part id and the terms are loaded together
                        // (all in bounds for any node id)
                        const i32 pu = A.part[u];
                        cv = make_int4(A.subk[u], A.cut[u], A.win[u],
                                       G.k[u] | (cyc[u] ? (i32)0x80000000 : 0));
                        if (pu != pid) {
                            S.cflag[i] = CF_GONE;
                            continue;
                        }
                        CV[i] = cv;
                        S.cflag[i] = 0;
                    } else {
                        cv = CV[i];
                    }
                    const i64 ku = cv.w & 0x7fffffff;
                    gm = min(gm, m2 * (i64)cv.z - ku * (sig - ku));
                    if (cv.w >= 0) {
                        const i64 sx = cv.x;
                        const i64 key = sx * (sig - sx) - m2 * (i64)cv.y;
                        const u64 pr = ((u64)(u32)u << 32) | (u64)(u32)u;
                        if (key > bk || (key == bk && pr < bp)) {
                            bk = key;
                            bp = pr;
                        }
                    }
                }
                neg = gm < 0 ? 1 : 0;
            }
            // cycle cuts: pairs p < q of cycle positions
            if (L >= 2) {
                for (int t = threadIdx.x; t < L * L; t += PW_BS) {
                    const int p = t / L, q = t % L;
                    if (q <= p) continue;
                    i64 sy = 0, wxy = 0;
                    for (int j = p + 1; j <= q; j++) {
                        sy += A.subk[CN[j]];
                        for (int l = 0; l < L; l++)
                            if (l <= p || l > q) wxy += Wm[j * L + l];
                    }
                    const i64 key = sy * (sig - sy) - m2 * wxy;
                    const i32 x = CN[p], y = CN[q];
                    const u64 pr = x < y ? (((u64)(u32)x << 32) | (u64)(u32)y)
                                         : (((u64)(u32)y << 32) | (u64)(u32)x);
                    if (key > bk || (key == bk && pr < bp)) {
                        bk = key;
                        bp = pr;
                    }
                }
            }
            wg_best_or(bk, bp, neg, S);
            if (!scanned) {
                // the set decides only if no node outside it can change the
                // answer; otherwise scan the whole part
                const i64 D = S.sig_scan - sig;
                u64 tpair;
                i64 thr, lb;
                pw_bounds(S, D, thr, tpair, lb);
                bool sure = true;
                if (!neg && lb < 0) sure = false;
                if (neg && bp != ~0ull && !(bk > thr || (bk == thr && bp < tpair))) sure = false;
                if (neg && bp == ~0ull && thr != INT64_MIN) sure = false;
                if (!sure) {
                    if (threadIdx.x == 0) S.need_scan = 1;
                    __syncthreads();
                    continue;
                }
            }
            if (!neg || bp == ~0ull) break;
            const i32 x = (i32)(bp >> 32), y = (i32)(bp & 0xffffffffu);
            if (threadIdx.x == 0) atomicAdd((unsigned long long *)A.splits, 1ull);
            if (x != y) {
                // ---------------- cycle cut: rebuild both sides
                int p = A.cpos[x], q = A.cpos[y];
                i32 cp = x, cq = y;
                if (p > q) {
                    int tt = p;
                    p = q;
                    q = tt;
                    cp = y;
                    cq = x;
                }
                __syncthreads();
                for (int j = threadIdx.x; j < L; j += PW_BS) cyc[CN[j]] = 0;
                __syncthreads();
                if (threadIdx.x == 0) {
                    cyc[x] = 1;
                    cyc[y] = 1;
                    a[x] = x;
                    a[y] = y;
                }
                const int pp = p, qq = q;
                auto inX = [&](i32 u) {
                    const int pr = A.cpos[A.root[u]];
                    return !(pr > pp && pr <= qq);
                };
                // the members still in the part first, then the two sides
                const int live =
                    wg_partition(P, m, ORD, [&](i32 u) { return A.part[u] == pid; }, S);
                const int nx = wg_partition(P, live, ORD, inX, S);
                // both sides take their ids now: a one-node side is never
                // rebuilt, and the other side must not count it as a member
                for (int i = threadIdx.x; i < live; i += PW_BS) A.part[P[i]] = i < nx ? cp : cq;
                __syncthreads();
                if (threadIdx.x == 0) {
                    pw_assign(STK, S.sp0, S.sp, s + live);
                    if (S.sp + 2 > m0) report(A.err, 10);
                    else {
                        STK[S.sp++] = make_int4(s, s + nx, cp, ST_INIT);
                        STK[S.sp++] = make_int4(s + nx, s + live, cq, ST_INIT);
                    }
                }
                __syncthreads();
                break;
            }
            // ---------------- branch cut at x: T_x leaves the part
            // (thread 0 writes below none of what the others read here)
            // every load that depends on x alone is issued here, before the
            // set-up barrier (which the compiler does not move loads across)
            const i32 px = a[x];
            const i32 rx = A.root[x];
            const i64 sx = A.subk[x];
            const bool leaf = A.chc[x] == 0;  // a node without children is T_x by itself
            const i64 rpx0 = G.rp[x], rpx1 = G.rp[x + 1];
            // x is no cycle node, so its parent is in the part one level up
            const int dpx = A.dep[x] - 1;
            // T_x in level order: TMP[0..t)
            if (threadIdx.x == 0) {
                TMP[0] = x;
                S.head = 0;
                S.tail = 1;
                S.lev_end = 1;
                A.part[x] = x;
                pw_drop_cand(S, x);
            }
            // a cut of a node without children goes on without a barrier:
            // its entry pass reads nothing that thread 0 writes here (it skips
            // x by id, and no path correction reaches a node without
            // children), and x's own root, parent and cycle mark, which other
            // threads may still be loading, are written after the split's last
            // barrier; leaf is the same in every thread
            if (!leaf) __syncthreads();
            while (!leaf) {
                const int lb = S.head, le = S.lev_end;
                if (lb == le) break;
                for (int i = lb + threadIdx.x; i < le; i += PW_BS) {
                    i32 u = TMP[i];
                    int c = A.chc[u];
                    int cs = A.chs[u];
                    for (int j = 0; j < c; j++) {
                        i32 ch = CHL[cs + j];
                        if (A.part[ch] != pid) continue;
                        int q = atomicAdd(&S.tail, 1);
                        TMP[q] = ch;
                        A.part[ch] = x;
                        pw_drop_cand(S, ch);
                    }
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    S.head = le;
                    S.lev_end = S.tail;
                }
                __syncthreads();
            }
            const int tcount = leaf ? 1 : S.tail;
            if (!leaf)
                for (int i = threadIdx.x; i < tcount; i += PW_BS) A.root[TMP[i]] = x;
            // The ancestors of x lose S_{T_x}; the last thread walks them while
            // the others take the entries below.  The two touch disjoint data:
            // the walk writes subk (and a[x] and cyc[x] when x has children),
            // and the entry pass reads
            // only nodes outside T_x and paths that never reach x (nothing
            // else there writes subk).  A cut of more than one node computes a
            // degree prefix first, whose barriers the walk precedes.
            if (threadIdx.x == PW_BS - 1) {
                i32 yv = px;
                for (int guard = 0;; guard++) {
                    if (guard >= m) {
                        report(A.err, 4);
                        break;
                    }
                    // the next ancestor and the cycle flag are loaded before
                    // the candidate add, whose atomic the walk then overlaps
                    const i32 ny = a[yv];
                    const bool top = cyc[yv] != 0;
                    A.subk[yv] -= (i32)sx;
                    pw_add_cand(S, yv);
                    if (top) break;
                    yv = ny;
                }
                if (!leaf) {
                    a[x] = x;
                    cyc[x] = 1;
                }
            }
            // entries between T_x and the rest of the part (a single node's
            // entries need no degree prefix)
            const i64 tot = tcount == 1 ? rpx1 - rpx0
                                        : wg_degree_prefix(TMP, tcount, G.rp, DP, S);
            for (i64 b = 0, sl = 0; b < tot; b += PW_BS) {
                const i64 t = b + threadIdx.x;
                int slot = 0, snx = 0;
                i64 d0 = 0;
                if (tcount > 1) wg_block_slot(DP, tcount, tot, b, (int)sl, slot, d0, snx, S);
                sl = snx;
                i32 v = 0;
                i64 val = 0;
                if (t < tot) {
                    v = tcount == 1 ? x : TMP[slot];
                    int2 ed = G.e[(tcount == 1 ? rpx0 : G.rp[v]) + (t - d0)];
                    i32 u = ed.x;
                    // u's part id, depth and parent in one round of loads
                    // (in bounds for any node id)
                    const i32 pu = A.part[u], au = a[u];
                    const int du = A.dep[u];
                    if (u != x && pu == pid) {
                        val = ed.y;
                        const i32 A_ = ed.y;
                        atomicSub(&A.win[u], A_);
                        pw_add_cand(S, u);
                        // paths u -> lca and px -> lca in the part before the
                        // cut.  Inside a part a parent is one level above its
                        // child, so the depths are counted down instead of
                        // loaded, and each step loads the next node before
                        // its candidate add
                        i32 p1 = u, p2 = px;
                        int d1 = du, d2 = dpx;
                        int guard = 0;
                        if (d1 > d2) {  // the first step up from u
                            guard++;
                            atomicSub(&A.cut[p1], A_);
                            pw_add_cand(S, p1);
                            p1 = au;
                            d1--;
                        }
                        while (d1 > d2 && guard++ < 2 * m) {
                            const i32 n1 = a[p1];
                            atomicSub(&A.cut[p1], A_);
                            pw_add_cand(S, p1);
                            p1 = n1;
                            d1--;
                        }
                        while (d2 > d1 && guard++ < 2 * m) {
                            const i32 n2 = a[p2];
                            atomicSub(&A.cut[p2], A_);
                            pw_add_cand(S, p2);
                            p2 = n2;
                            d2--;
                        }
                        while (p1 != p2 && guard++ < 2 * m) {
                            const i32 n1 = a[p1], n2 = a[p2];
                            const bool top = cyc[p1] && cyc[p2];
                            atomicSub(&A.cut[p1], A_);
                            atomicSub(&A.cut[p2], A_);
                            pw_add_cand(S, p1);
                            pw_add_cand(S, p2);
                            if (top) break;
                            p1 = n1;
                            p2 = n2;
                        }
                        if (guard >= 2 * m) report(A.err, 2);
                        // path v -> x inside T_x
                        guard = 0;
                        for (i32 q = v; q != x && guard < m; q = a[q], guard++)
                            atomicSub(&A.cut[q], A_);
                        if (guard >= m) report(A.err, 3);
                        if (L >= 2 && A.root[u] != rx) {
                            const int j = A.cpos[rx], l = A.cpos[A.root[u]];
                            atomicAdd((unsigned long long *)&Wm[j * L + l], (unsigned long long)(-(i64)A_));
                            atomicAdd((unsigned long long *)&Wm[l * L + j], (unsigned long long)(-(i64)A_));
                        }
                    }
                }
                wave_run_add(t < tot, v, -val, A.win);
            }
            // T_x stays in the range, marked by its id, and waits on the stack
            // for a range of its own (a single node needs none); nothing in
            // the pass reads S.sp or S.sig.  A candidate set that overflowed
            // in this pass makes the next pass scan (read at its start).
            if (threadIdx.x == 0) {
                if (tcount > 1) {
                    if (S.sp >= m0) report(A.err, 10);
                    else STK[S.sp++] = make_int4(-1, tcount, x, ST_GATHER);
                }
                S.sig = sig - sx;
            }
            __syncthreads();
            if (leaf && threadIdx.x == 0) {
                A.root[x] = x;
                a[x] = x;
                cyc[x] = 1;
            }
        }
        // the subtrees cut off this part take their ranges inside it
        if (threadIdx.x == 0) pw_assign(STK, S.sp0, S.sp, s);
        __syncthreads();
    }
}


void launch_positive_wg(const PosArgs &A, i64 nflag, hipStream_t s)
{
    if (nflag > 0) k_positive_wg<<<(unsigned)nflag, PW_BS, 0, s>>>(A);
}
