// POSITIVE (Sec. 3.3, appendix POSITIVE) under the directed model, where a
// node carries two strengths x and y (the null-model term of merging node
// sets P and R is X_P X_R - Y_P Y_R).  One workgroup per community holding a
// node of negative local gain runs the while loop of the appendix POSITIVE
// plainly: it keeps a stack of parts (ranges of the community's member
// list); for the part on top it computes the local gains
//     g(u) = A w(u, P \ u) - x_u (X_P - x_u) + y_u (Y_P - y_u)
// and, when one is negative, the part's cycle, its hanging trees in DFS
// order with their subtree sums, and every bisection from scratch:
//     branch x      X_T (X_P - X_T) - Y_T (Y_P - Y_T) - A cut(T),  T = T_x
//     cycle (p, q)  the same with T = the hanging trees at cycle positions
//                   p+1..q (the side rooted at the q-th cycle node)
// ties to the lowest (first, second) cut node.  The best cut is applied
// (self-assignments) and both sides go back on the stack.  Part ids are
// node ids of the part itself, so they never collide with another part's.
//
// The undirected model runs k_positive_wg, whose incremental split search
// relies on keys that only fall as X_P falls; with a y term that no longer
// bounds them, so this kernel re-evaluates every cut at every split.
#include "slm_forest.h"

#define PD_BS 256
#define PD_NW (PD_BS / 64)

struct PdShared {
    i64 red[2 * PD_NW];
    int redf[PD_NW];
    int sp;      // stack size
    int stop;    // the stack was empty at the last pop
    int s, e, pid;
    int L;       // cycle length of the part (-1: inconsistent)
    i32 cyc0;    // smallest cycle node
    int na;      // size of the first side after a split
    i32 pida, pidb;
};

__device__ __forceinline__ void pd_report(int *err, int code)
{
    atomicCAS(err, 0, code);
}

__device__ __forceinline__ i64 pd_sum(i64 v, PdShared &S)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wid = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) S.red[wid] = v;
    __syncthreads();
    i64 t = 0;
    for (int w = 0; w < PD_NW; w++) t += S.red[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ int pd_or(int f, PdShared &S)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) f |= __shfl_xor(f, off, 64);
    const int wid = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) S.redf[wid] = f;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < PD_NW; w++) t |= S.redf[w];
    __syncthreads();
    return t;
}

// Largest key, ties to the lowest pair, over the workgroup.
__device__ __forceinline__ void pd_best(i64 &key, u64 &pair, PdShared &S)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const i64 ok = __shfl_xor(key, off, 64);
        const u64 op = __shfl_xor(pair, off, 64);
        if (ok > key || (ok == key && op < pair)) {
            key = ok;
            pair = op;
        }
    }
    const int wid = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        S.red[2 * wid] = key;
        S.red[2 * wid + 1] = (i64)pair;
    }
    __syncthreads();
    key = S.red[0];
    pair = (u64)S.red[1];
    for (int w = 1; w < PD_NW; w++) {
        const i64 k2 = S.red[2 * w];
        const u64 p2 = (u64)S.red[2 * w + 1];
        if (k2 > key || (k2 == key && p2 < pair)) {
            key = k2;
            pair = p2;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void pd_consider(i64 key, i32 f, i32 s, i64 &bk, u64 &bp)
{
    const u64 pr = ((u64)(u32)f << 32) | (u64)(u32)s;
    if (key > bk || (key == bk && pr < bp)) {
        bk = key;
        bp = pr;
    }
}

__global__ __launch_bounds__(PD_BS) void k_positive_dir(PosArgs A)
{
    __shared__ PdShared S;
    const int f = blockIdx.x;
    const i64 base = A.mem_off[f];
    const int m0 = (int)(A.mem_off[f + 1] - base);
    i32 *M = A.mem + base;         // the community's members; parts are ranges
    i32 *TMP = A.tmp + base;       // DFS stack and partition scratch (m0)
    i32 *ORD = A.ord + base;       // DFS order of the current part (m0)
    i32 *CHL = A.chl + 2 * base;   // children lists of the current part (m0)
    int4 *STK = A.stk + base;      // part stack (at most m0 entries)
    const int Lc0 = A.lcyc[f];     // cycle length of the community; no part's is longer
    i64 *Wt = Lc0 >= 2 ? A.W + A.woff[f] : nullptr;  // Lc0 x Lc0 tree-to-tree weights
    i32 *CN = Lc0 >= 2 ? A.cn + A.noff[f] : nullptr;  // cycle nodes in pointer order
    const LevelView &G = A.G;
    const i64 Asc = node_m2(G, M[0]);
    i32 *a = A.a;
    uint8_t *cyc = A.cyc;
    i32 *tin = A.dep, *tout = A.root, *cur = A.win;
    i32 *sub = A.subk, *suby = A.cut;  // subtree sums of x and of y
    const int cap = 4 * m0 + 16;       // pops: a part is split at most m0 - 1 times

    if (threadIdx.x == 0) {
        STK[0] = make_int4(0, m0, A.flist[f], 0);
        S.sp = 1;
    }
    __syncthreads();
    int iters = 0;
    while (true) {
        // thread 0 pops between two barriers; every thread decides from the
        // record it leaves, never from the stack size
        __syncthreads();
        if (threadIdx.x == 0) {
            S.stop = S.sp == 0;
            if (!S.stop) {
                const int4 t = STK[--S.sp];
                S.s = t.x;
                S.e = t.y;
                S.pid = t.z;
            }
        }
        __syncthreads();
        if (S.stop) break;
        if (++iters > cap) {
            if (threadIdx.x == 0) pd_report(A.err, 5);
            break;
        }
        const int s = S.s, e = S.e, pid = S.pid;
        if (s < 0 || e < s || e > m0) {
            if (threadIdx.x == 0) pd_report(A.err, 9);
            break;
        }
        const int m = e - s;
        i32 *P = M + s;
        if (m <= 1) {
            if (m == 1 && threadIdx.x == 0) A.part[P[0]] = pid;
            continue;
        }
        // ---------------------------------------------- part ids, totals, gains
        i64 sx = 0, sy = 0;
        for (int i = threadIdx.x; i < m; i += PD_BS) {
            const i32 u = P[i];
            A.part[u] = pid;
            sx += G.k[u];
            sy += node_y(G, u);
        }
        sx = pd_sum(sx, S);  // its barriers also publish the part ids
        sy = pd_sum(sy, S);
        int neg = 0;
        for (int i = threadIdx.x; i < m; i += PD_BS) {
            const i32 u = P[i];
            i64 win = 0;
            for (i64 j = G.rp[u]; j < G.rp[u + 1]; j++) {
                const int2 ed = G.e[j];
                if (ed.x != u && A.part[ed.x] == pid) win += ed.y;
            }
            const i64 xu = G.k[u], yu = node_y(G, u);
            if (Asc * win - xu * (sx - xu) + yu * (sy - yu) < 0) neg = 1;
        }
        neg = pd_or(neg, S);
        if (!neg) continue;
        // ---------------------------------------------- the cycle (thread 0)
        if (threadIdx.x == 0) {
            i32 x = P[0];
            for (int t = 0; t < m; t++) x = a[x];  // m steps reach the cycle
            int L = 0;
            i32 y = x, mn = x;
            do {
                L++;
                if (y < mn) mn = y;
                y = a[y];
            } while (y != x && L <= m);
            if (y != x || (L >= 2 && L > Lc0)) {
                pd_report(A.err, 10);
                L = -1;
            }
            S.L = L;
            S.cyc0 = mn;
            if (L >= 2) {
                y = mn;
                for (int t = 0; t < L; t++) {
                    CN[t] = y;
                    y = a[y];
                }
            }
        }
        __syncthreads();
        const int L = S.L;
        if (L < 0) break;
        // ---------------------------------------------- forest of the part
        for (int i = threadIdx.x; i < m; i += PD_BS) {
            const i32 u = P[i];
            cyc[u] = 0;
            A.chc[u] = 0;
            sub[u] = G.k[u];
            suby[u] = (i32)node_y(G, u);
        }
        __syncthreads();
        if (L == 1) {
            if (threadIdx.x == 0) cyc[S.cyc0] = 1;
        } else {
            for (int t = threadIdx.x; t < L; t += PD_BS) cyc[CN[t]] = 1;
        }
        __syncthreads();
        // (a parent outside the part would mean an inconsistent part: such a
        // child is left out, the DFS then misses it and reports the part)
        for (int i = threadIdx.x; i < m; i += PD_BS) {
            const i32 u = P[i];
            if (!cyc[u] && A.part[a[u]] == pid) atomicAdd(&A.chc[a[u]], 1);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int off = 0;
            for (int i = 0; i < m; i++) {
                const i32 u = P[i];
                A.chs[u] = off;
                off += A.chc[u];
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += PD_BS) cur[P[i]] = A.chs[P[i]];
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += PD_BS) {
            const i32 u = P[i];
            if (!cyc[u] && A.part[a[u]] == pid) CHL[atomicAdd(&cur[a[u]], 1)] = u;
        }
        __syncthreads();
        // DFS from every cycle node in cycle order, then subtree sums in
        // reverse DFS order (children come after their parent)
        if (threadIdx.x == 0) {
            for (int i = 0; i < m; i++) cur[P[i]] = A.chs[P[i]];
            int t = 0;
            for (int p = 0; p < L; p++) {
                const i32 r = L == 1 ? S.cyc0 : CN[p];
                int sp = 0;
                TMP[sp++] = r;
                tin[r] = t;
                ORD[t++] = r;
                A.cpos[r] = p;
                while (sp > 0 && t <= m) {
                    const i32 u = TMP[sp - 1];
                    if (cur[u] < A.chs[u] + A.chc[u]) {
                        const i32 c = CHL[cur[u]++];
                        tin[c] = t;
                        if (t < m) ORD[t] = c;
                        t++;
                        A.cpos[c] = p;
                        TMP[sp++] = c;
                    } else {
                        tout[u] = t;
                        sp--;
                    }
                }
            }
            if (t != m) {
                pd_report(A.err, 11);  // the part is not one component
                S.L = -1;
            } else {
                for (int q = m - 1; q >= 0; q--) {
                    const i32 u = ORD[q];
                    if (!cyc[u]) {
                        sub[a[u]] += sub[u];
                        suby[a[u]] += suby[u];
                    }
                }
            }
        }
        __syncthreads();
        if (S.L < 0) break;
        // ---------------------------------------------- branch cuts
        i64 bk = INT64_MIN;
        u64 bp = ~0ull;
        for (int i = threadIdx.x; i < m; i += PD_BS) {
            const i32 x = P[i];
            if (cyc[x]) continue;
            const int t0 = tin[x], t1 = tout[x];
            i64 cut = 0;
            for (int t = t0; t < t1; t++) {
                const i32 u = ORD[t];
                for (i64 j = G.rp[u]; j < G.rp[u + 1]; j++) {
                    const int2 ed = G.e[j];
                    if (A.part[ed.x] != pid) continue;
                    const int tv = tin[ed.x];
                    if (tv < t0 || tv >= t1) cut += ed.y;
                }
            }
            const i64 X = sub[x], Y = suby[x];
            pd_consider(X * (sx - X) - Y * (sy - Y) - Asc * cut, x, x, bk, bp);
        }
        // ---------------------------------------------- cycle cuts
        if (L >= 2) {
            for (int t = threadIdx.x; t < L * L; t += PD_BS) Wt[t] = 0;
            __syncthreads();
            for (int i = threadIdx.x; i < m; i += PD_BS) {
                const i32 u = P[i];
                const int pu = A.cpos[u];
                for (i64 j = G.rp[u]; j < G.rp[u + 1]; j++) {
                    const int2 ed = G.e[j];
                    if (A.part[ed.x] != pid) continue;
                    atomicAdd((unsigned long long *)&Wt[(i64)pu * L + A.cpos[ed.x]],
                              (unsigned long long)(i64)ed.y);
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {  // inclusive 2-D prefix sums
                for (int r = 0; r < L; r++)
                    for (int c = 0; c < L; c++) {
                        i64 v = Wt[(i64)r * L + c];
                        if (r) v += Wt[(i64)(r - 1) * L + c];
                        if (c) v += Wt[(i64)r * L + c - 1];
                        if (r && c) v -= Wt[(i64)(r - 1) * L + c - 1];
                        Wt[(i64)r * L + c] = v;
                    }
            }
            __syncthreads();
            const int npair = L * (L - 1) / 2;
            for (int q = threadIdx.x; q < npair; q += PD_BS) {
                int p = 0, rest = q;
                while (rest >= L - 1 - p) {
                    rest -= L - 1 - p;
                    p++;
                }
                const int r = p + 1 + rest;  // positions p < r; T = (p, r]
                i64 X = 0, Y = 0;
                for (int t = p + 1; t <= r; t++) {
                    X += sub[CN[t]];
                    Y += suby[CN[t]];
                }
                const i64 rows = Wt[(i64)r * L + L - 1] - Wt[(i64)p * L + L - 1];
                const i64 blk = Wt[(i64)r * L + r] - Wt[(i64)p * L + r] - Wt[(i64)r * L + p] +
                                Wt[(i64)p * L + p];
                const i64 cut = rows - blk;
                const i32 x = CN[p], y = CN[r];
                pd_consider(X * (sx - X) - Y * (sy - Y) - Asc * cut, x < y ? x : y, x < y ? y : x,
                            bk, bp);
            }
        }
        pd_best(bk, bp, S);
        const i32 c1 = (i32)(bp >> 32), c2 = (i32)(u32)bp;
        // ---------------------------------------------- apply, split the range
        if (threadIdx.x == 0) {
            int na = 0;
            if (c1 == c2) {
                // branch: T_x first, then the rest (which keeps the cycle)
                const int t0 = tin[c1], t1 = tout[c1];
                for (int i = 0; i < m; i++)
                    if (tin[P[i]] >= t0 && tin[P[i]] < t1) TMP[na++] = P[i];
                int k = na;
                for (int i = 0; i < m; i++)
                    if (!(tin[P[i]] >= t0 && tin[P[i]] < t1)) TMP[k++] = P[i];
                a[c1] = c1;
                cyc[c1] = 1;
                S.pida = c1;
                S.pidb = L == 1 ? S.cyc0 : CN[0];
            } else {
                // cycle: the side rooted at the later position first
                int p = A.cpos[c1], r = A.cpos[c2];
                if (p > r) {
                    const int t = p;
                    p = r;
                    r = t;
                }
                for (int i = 0; i < m; i++) {
                    const int t = A.cpos[P[i]];
                    if (t > p && t <= r) TMP[na++] = P[i];
                }
                int k = na;
                for (int i = 0; i < m; i++) {
                    const int t = A.cpos[P[i]];
                    if (!(t > p && t <= r)) TMP[k++] = P[i];
                }
                for (int t = 0; t < L; t++) cyc[CN[t]] = 0;
                a[CN[p]] = CN[p];
                a[CN[r]] = CN[r];
                cyc[CN[p]] = 1;
                cyc[CN[r]] = 1;
                S.pida = CN[r];
                S.pidb = CN[p];
            }
            S.na = na;
            atomicAdd((unsigned long long *)A.splits, 1ull);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += PD_BS) P[i] = TMP[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            if (S.na < 1 || S.na >= m || S.sp + 2 > m0) {
                pd_report(A.err, 12);
                S.sp = 0;
            } else {
                STK[S.sp++] = make_int4(s + S.na, e, S.pidb, 0);
                STK[S.sp++] = make_int4(s, s + S.na, S.pida, 0);
            }
        }
        __syncthreads();
    }
}

void launch_positive_dir(const PosArgs &A, i64 nflag, hipStream_t s)
{
    if (nflag > 0) k_positive_dir<<<(unsigned)nflag, PD_BS, 0, s>>>(A);
}
