// Classical Louvain local moving (the sequential method the SLM builds on,
// named in Sec. 6 as the comparison left open) with its exact sequential
// result on the GPU.  In id order, node i moves to its best neighbouring
// community C (join(i,C) = M2 w(i,C) - k_i S_C, lowest name on ties) when
// that beats stay(i) = M2 w(i, c\i) - k_i (S_c - k_i), seeing every move made
// before it.  Communities are named by the node they started from.
//
// Speculation by chunks.  The next B nodes decide at once from the state at
// the chunk's start.  Node i's decision reads the names of its neighbours and
// the totals S of its own and its neighbours' communities; a move of node j
// writes j's name and the totals of j's old and new communities.  Every
// moving node marks what it writes with its position in the chunk (atomic
// min), so node i is exact if no earlier mover of the chunk marked anything
// i reads.  A node whose neighbours kept their names but some of whose
// communities' totals changed is still exact when its decision holds for
// every value those totals can have: each such total lies between its value
// at the chunk's start less the strengths of the chunk's movers out of the
// community and plus those of its movers into it (all strengths are
// non-negative), and the chosen option must beat every other one strictly
// over that box.  The moves before the first node that is not exact are
// applied -- exactly the sequential result -- and the next chunk starts at
// that node.  The first node of a chunk is always exact, so every chunk makes
// progress.
#include "slm_forest.h"

#define LV_BS 256
#define LV_NODES (LV_BS / 64)  // one wavefront per node
#define LV_BMIN 64
#define LV_BMAX 16384
#define LV_BATCH 16            // chunks launched between two host reads
#define LV_LT 1024             // LDS table slots per wavefront (rows of degree <= 512)

// Chunk state on the device, so that the GPU moves from chunk to chunk
// without the host: the chunk is [p, p + min(B, n - p)); first = the first
// position whose decision read something an earlier mover of the chunk wrote;
// err = a chunk made no progress.  Kernels of a chunk that starts at or past
// n do nothing, so the host can launch several chunks ahead of its reads.
struct LvState {
    i64 p, B;
    int first, err;
};

__device__ __forceinline__ i64 lv_count(const LvState *st, i64 n)
{
    const i64 p = st->p;
    if (p >= n) return 0;
    return st->B < n - p ? st->B : n - p;
}

// The decision of node i = p + t from w(i, c_i \ i) and its best neighbouring
// community (bk, bc): dest[t] = the community to move to, or -1; win[t] =
// w(i, c_i \ i).  A moving node marks its own name and the totals of its old
// and new communities with t, and adds its strength to the chunk's movers out
// of its old community (kout) and into its new one (kin).
__device__ __forceinline__ void lv_finish(i64 t, i64 i, i32 ci, i64 ki, i64 m2, i64 w_in, i64 bk,
                                          i32 bc, const i32 *__restrict__ sig,
                                          i32 *__restrict__ dest, i32 *__restrict__ win,
                                          i32 *__restrict__ mark_node, i32 *__restrict__ mark_comm,
                                          i32 *__restrict__ kin, i32 *__restrict__ kout)
{
    const i64 stay = m2 * w_in - ki * ((i64)sig[ci] - ki);
    const bool mv = bc != INT32_MAX && bk > stay;
    dest[t] = mv ? bc : -1;
    win[t] = (i32)w_in;
    if (mv) {
        atomicMin(&mark_node[i], (i32)t);
        atomicMin(&mark_comm[ci], (i32)t);
        atomicMin(&mark_comm[bc], (i32)t);
        atomicAdd(&kout[ci], (i32)ki);
        atomicAdd(&kin[bc], (i32)ki);
    }
}

// Node i = p + t of the chunk decides from the current names c[] and totals
// sig[], with a hash table of its neighbours' communities of twice its
// degree in slots: rows of degree <= LV_LT / 2 in their wavefront's LDS
// table, rows of degree <= LV_NODES * LV_LT / 2 one after another by the
// whole workgroup in the LDS of all four, longer rows in global memory.
// Either way the table ends at the row's global slots [2 (rp[i] - rp[p]),
// 2 (rp[i+1] - rp[p])) for the conflict check.
__global__ __launch_bounds__(LV_BS) void k_lv_decide(LevelView L, const LvState *__restrict__ st,
                                                    const i32 *__restrict__ c,
                                                    const i32 *__restrict__ sig,
                                                    i32 *__restrict__ tkey,
                                                    i32 *__restrict__ tval,
                                                    i32 *__restrict__ dest,
                                                    i32 *__restrict__ win,
                                                    i32 *__restrict__ mark_node,
                                                    i32 *__restrict__ mark_comm,
                                                    i32 *__restrict__ kin,
                                                    i32 *__restrict__ kout)
{
    __shared__ i32 lkey[LV_NODES][LV_LT];
    __shared__ i32 lval[LV_NODES][LV_LT];
    __shared__ i64 red[2 * LV_NODES];
    const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
    const i64 cnt = lv_count(st, L.n);
    const i64 blk0 = (i64)blockIdx.x * LV_NODES;
    if (blk0 >= cnt) return;  // the whole workgroup leaves together
    const i64 p = st->p;
    const i64 rp0 = L.rp[p];
    const i64 m2 = L.m2;
    const i64 t = blk0 + wid;
    if (t < cnt) {
        const i64 i = p + t;
        const i64 e0 = L.rp[i], e1 = L.rp[i + 1];
        const i64 H = 2 * (e1 - e0);
        const i64 tb = 2 * (e0 - rp0);
        const i32 ci = c[i];
        const i64 ki = L.k[i];
        i64 w_in = 0;
        i64 bk = INT64_MIN;
        i32 bc = INT32_MAX;
        if (H <= LV_LT) {
            // the wavefront's table in LDS, copied out for the conflict check
            for (int h = lane; h < (int)H; h += 64) {
                lkey[wid][h] = -1;
                lval[wid][h] = 0;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (i64 j = e0 + lane; j < e1; j += 64) {
                const int2 ed = L.e[j];
                if (ed.x == i) continue;
                const i32 cv = c[ed.x];
                if (cv == ci) {
                    w_in += ed.y;
                    continue;
                }
                u32 h = (u32)(((u64)hash_label(cv) * (u64)H) >> 32);
                for (int probe = 0; probe < (int)H; probe++) {
                    const i32 old = atomicCAS(&lkey[wid][h], -1, cv);
                    if (old == -1 || old == cv) {
                        atomicAdd(&lval[wid][h], ed.y);
                        break;
                    }
                    h = h + 1 == (u32)H ? 0u : h + 1;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (int h = lane; h < (int)H; h += 64) {
                const i32 cc = lkey[wid][h];
                const i32 wv = lval[wid][h];
                tkey[tb + h] = cc;
                tval[tb + h] = wv;
                if (cc < 0) continue;
                const i64 key = m2 * (i64)wv - ki * (i64)sig[cc];
                if (better_key(key, cc, bk, bc)) {
                    bk = key;
                    bc = cc;
                }
            }
        } else if (H > LV_NODES * LV_LT) {
            i32 *keys = tkey + tb;
            i32 *vals = tval + tb;
            for (i64 h = lane; h < H; h += 64) {
                keys[h] = -1;
                vals[h] = 0;
            }
            // the cleared slots are visible to the wavefront's inserts
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            __builtin_amdgcn_wave_barrier();
            for (i64 j = e0 + lane; j < e1; j += 64) {
                const int2 ed = L.e[j];
                if (ed.x == i) continue;
                const i32 cv = c[ed.x];
                if (cv == ci) {
                    w_in += ed.y;
                    continue;
                }
                u64 h = ((u64)hash_label(cv) * (u64)H) >> 32;
                for (i64 probe = 0; probe < H; probe++) {
                    const i32 old = atomicCAS(&keys[h], -1, cv);
                    if (old == -1 || old == cv) {
                        atomicAdd(&vals[h], ed.y);
                        break;
                    }
                    h = h + 1 == (u64)H ? 0 : h + 1;
                }
            }
            // every insert of the wavefront is done and visible before the read-out
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
            __builtin_amdgcn_wave_barrier();
            for (i64 h = lane; h < H; h += 64) {
                const i32 cc =
                    __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (cc < 0) continue;
                const i32 wv =
                    __hip_atomic_load(&vals[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const i64 key = m2 * (i64)wv - ki * (i64)sig[cc];
                if (better_key(key, cc, bk, bc)) {
                    bk = key;
                    bc = cc;
                }
            }
        }
        if (H <= LV_LT || H > LV_NODES * LV_LT) {
            w_in = group_sum<64, i64>(w_in);
            group_best<64>(bk, bc);
            if (lane == 0)
                lv_finish(t, i, ci, ki, m2, w_in, bk, bc, sig, dest, win, mark_node, mark_comm,
                          kin, kout);
        }
    }
    // the workgroup's medium-long rows, one after another, in one LDS table
    // of LV_NODES * LV_LT slots (every thread reads the same row sizes, so
    // the loop and its barriers are uniform)
    i32 *fk = &lkey[0][0];
    i32 *fv = &lval[0][0];
    for (int q = 0; q < LV_NODES; q++) {
        const i64 tq = blk0 + q;
        if (tq >= cnt) break;
        const i64 i = p + tq;
        const i64 e0 = L.rp[i], e1 = L.rp[i + 1];
        const i64 H = 2 * (e1 - e0);
        if (H <= LV_LT || H > LV_NODES * LV_LT) continue;
        const i64 tb = 2 * (e0 - rp0);
        const i32 ci = c[i];
        const i64 ki = L.k[i];
        __syncthreads();  // the tables of the previous row (or of the wavefronts) are done
        for (int h = threadIdx.x; h < (int)H; h += LV_BS) {
            fk[h] = -1;
            fv[h] = 0;
        }
        __syncthreads();
        i64 w_in = 0;
        for (i64 j = e0 + threadIdx.x; j < e1; j += LV_BS) {
            const int2 ed = L.e[j];
            if (ed.x == i) continue;
            const i32 cv = c[ed.x];
            if (cv == ci) {
                w_in += ed.y;
                continue;
            }
            u32 h = (u32)(((u64)hash_label(cv) * (u64)H) >> 32);
            for (int probe = 0; probe < (int)H; probe++) {
                const i32 old = atomicCAS(&fk[h], -1, cv);
                if (old == -1 || old == cv) {
                    atomicAdd(&fv[h], ed.y);
                    break;
                }
                h = h + 1 == (u32)H ? 0u : h + 1;
            }
        }
        __syncthreads();
        i64 bk = INT64_MIN;
        i32 bc = INT32_MAX;
        for (int h = threadIdx.x; h < (int)H; h += LV_BS) {
            const i32 cc = fk[h];
            const i32 wv = fv[h];
            tkey[tb + h] = cc;
            tval[tb + h] = wv;
            if (cc < 0) continue;
            const i64 key = m2 * (i64)wv - ki * (i64)sig[cc];
            if (better_key(key, cc, bk, bc)) {
                bk = key;
                bc = cc;
            }
        }
        w_in = block_sum<i64>(w_in, red);
        block_best(bk, bc, red);
        if (threadIdx.x == 0)
            lv_finish(tq, i, ci, ki, m2, w_in, bk, bc, sig, dest, win, mark_node, mark_comm, kin,
                      kout);
    }
}

__device__ __forceinline__ i64 lv_wave_max(i64 v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const i64 o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Range of community C's total as node t of the chunk sees it: its value at
// the chunk's start when no earlier mover marked it, else that value less
// the chunk's movers out of C and plus its movers into C.
__device__ __forceinline__ void lv_total_range(i32 C, i64 t, const i32 *__restrict__ sig,
                                               const i32 *__restrict__ mark_comm,
                                               const i32 *__restrict__ kin,
                                               const i32 *__restrict__ kout, i64 &lo, i64 &hi)
{
    const i64 s0 = sig[C];
    lo = hi = s0;
    if (mark_comm[C] < t) {
        lo = s0 - kout[C];
        hi = s0 + kin[C];
    }
}

// first = the smallest t whose decision may differ from the one it would
// take after the chunk's earlier moves (it starts at INT32_MAX): a neighbour
// that moved earlier in the chunk, or a total that changed and could change
// the decision (the box test of the file header).
__global__ __launch_bounds__(LV_BS) void k_lv_conflict(LevelView L, LvState *__restrict__ st,
                                                      const i32 *__restrict__ c,
                                                      const i32 *__restrict__ sig,
                                                      const i32 *__restrict__ tkey,
                                                      const i32 *__restrict__ tval,
                                                      const i32 *__restrict__ dest,
                                                      const i32 *__restrict__ win,
                                                      const i32 *__restrict__ mark_node,
                                                      const i32 *__restrict__ mark_comm,
                                                      const i32 *__restrict__ kin,
                                                      const i32 *__restrict__ kout)
{
    const int lane = threadIdx.x & 63;
    const i64 cnt = lv_count(st, L.n);
    const i64 t = (i64)blockIdx.x * LV_NODES + threadIdx.x / 64;
    if (t >= cnt) return;
    const i64 p = st->p;
    const i64 i = p + t;
    const i32 ci = c[i];
    const i64 e0 = L.rp[i], e1 = L.rp[i + 1];
    bool moved_nb = false, changed = lane == 0 && mark_comm[ci] < t;
    for (i64 j = e0 + lane; j < e1; j += 64) {
        const i32 v = L.e[j].x;
        if (v == i) continue;
        if (mark_node[v] < t) moved_nb = true;
        if (mark_comm[c[v]] < t) changed = true;
    }
    if (__ballot(moved_nb) != 0) {
        if (lane == 0) atomicMin(&st->first, (int)t);
        return;
    }
    if (__ballot(changed) == 0) return;  // read nothing an earlier mover wrote
    // the decision must hold over the box of the changed totals
    const i64 ki = L.k[i], m2 = L.m2;
    const i32 d = dest[t];
    i64 lo, hi;
    lv_total_range(ci, t, sig, mark_comm, kin, kout, lo, hi);
    const i64 wi = win[t];
    const i64 stay_lo = m2 * wi - ki * (hi - ki), stay_hi = m2 * wi - ki * (lo - ki);
    const i64 H = 2 * (e1 - e0);
    const i64 tb = 2 * (e0 - L.rp[p]);
    i64 other_hi = INT64_MIN, d_lo = INT64_MIN;
    for (i64 h = lane; h < H; h += 64) {
        const i32 cc = tkey[tb + h];
        if (cc < 0) continue;
        const i64 wv = tval[tb + h];
        lv_total_range(cc, t, sig, mark_comm, kin, kout, lo, hi);
        if (cc == d) d_lo = m2 * wv - ki * hi;
        else other_hi = max(other_hi, m2 * wv - ki * lo);
    }
    other_hi = lv_wave_max(other_hi);
    d_lo = lv_wave_max(d_lo);
    const bool holds = d < 0 ? other_hi <= stay_lo : (d_lo > stay_hi && d_lo > other_hi);
    if (!holds && lane == 0) atomicMin(&st->first, (int)t);
}

// Applies the moves before `first` and clears every mark and mover sum of
// the chunk.
__global__ __launch_bounds__(LV_BS) void k_lv_apply(LevelView L, const LvState *__restrict__ st,
                                                   const i32 *__restrict__ dest,
                                                   i32 *__restrict__ c, i32 *__restrict__ sig,
                                                   i32 *__restrict__ mark_node,
                                                   i32 *__restrict__ mark_comm,
                                                   i32 *__restrict__ kin, i32 *__restrict__ kout,
                                                   unsigned long long *__restrict__ moves)
{
    const i64 cnt = lv_count(st, L.n);
    const i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const i32 d = dest[t];
    if (d < 0) return;
    const i64 i = st->p + t;
    const i32 old = c[i];
    mark_node[i] = INT32_MAX;
    mark_comm[old] = INT32_MAX;
    mark_comm[d] = INT32_MAX;
    kout[old] = 0;
    kin[d] = 0;
    if (t < (i64)st->first) {
        c[i] = d;
        atomicSub(&sig[old], L.k[i]);
        atomicAdd(&sig[d], L.k[i]);
        atomicAdd(moves, 1ull);
    }
}

// The next chunk starts at the first node that was not exact; the chunk size
// grows while whole chunks hold and shrinks when they break early.
__global__ void k_lv_advance(i64 n, LvState *__restrict__ st)
{
    if (st->p >= n) return;
    const i64 cnt = lv_count(st, n);
    const i64 done = st->first < cnt ? st->first : cnt;
    if (done < 1) {
        st->err = 1;
        st->p = n;  // the pass stops; the host reports the error
        return;
    }
    st->p += done;
    if (done == cnt && st->B < LV_BMAX) st->B *= 2;
    else if (done < cnt / 4 && st->B > LV_BMIN) st->B /= 2;
    st->first = INT32_MAX;
}

// A pass starts at node 0 (the chunk size carries over).
__global__ void k_lv_pass_start(LvState *__restrict__ st, unsigned long long *__restrict__ moves,
                                int reset_b)
{
    st->p = 0;
    if (reset_b) st->B = 1024;
    st->first = INT32_MAX;
    st->err = 0;
    *moves = 0;
}

// c[i] = i, sig[i] = k_i, no marks, no movers.
__global__ void k_lv_init(LevelView L, i32 *__restrict__ c, i32 *__restrict__ sig,
                          i32 *__restrict__ mark_node, i32 *__restrict__ mark_comm,
                          i32 *__restrict__ kin, i32 *__restrict__ kout)
{
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < L.n;
         i += (i64)gridDim.x * blockDim.x) {
        c[i] = (i32)i;
        sig[i] = L.k[i];
        mark_node[i] = INT32_MAX;
        mark_comm[i] = INT32_MAX;
        kin[i] = 0;
        kout[i] = 0;
    }
}

static unsigned lv_grid(i64 items, int per_block)
{
    i64 g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

// One level of local moving on the level in L; W.comp gets the community
// names.  Returns the passes that moved a node; *converged = the last pass
// moved nothing; *moves = nodes moved.  Tables use W.rk0 / W.rk1 (2 nnz int32
// slots each), names and totals W.comp / W.sigma, decisions W.best_c, marks
// W.M0 / W.M1, w(i, c_i \ i) of the chunk's nodes W.wc, the movers' sums
// W.A0 (into) / W.A1 (out of), the chunk state W.counters[2..4] and the move count
// W.counters[0].  The host launches LV_BATCH chunks at a time and reads the
// chunk state after each batch.
int louvain_level(Work &W, const LevelView &L, int max_passes, int *converged, i64 *moves,
                  hipStream_t s)
{
    const i64 n = L.n;
    i32 *c = W.comp, *sig = W.sigma, *dest = W.best_c, *mn = W.M0, *mc = W.M1;
    i32 *win = W.wc, *kin = W.A0, *kout = W.A1;
    i32 *tkey = (i32 *)W.rk0, *tval = (i32 *)W.rk1;
    unsigned long long *mv = (unsigned long long *)W.counters;
    LvState *st = (LvState *)(W.counters + 2);
    static_assert(sizeof(LvState) <= 3 * sizeof(i64), "chunk state must fit three counters");
    *converged = 0;
    *moves = 0;
    if (n == 0) {
        *converged = 1;
        return 0;
    }
    k_lv_init<<<lv_grid(n, SLM_BS) > 4096 ? 4096 : lv_grid(n, SLM_BS), SLM_BS, 0, s>>>(
        L, c, sig, mn, mc, kin, kout);
    const i64 bmax = n < LV_BMAX ? n : LV_BMAX;
    int passes = 0;
    while (passes < max_passes) {
        k_lv_pass_start<<<1, 1, 0, s>>>(st, mv, passes == 0);
        while (true) {
            for (int b = 0; b < LV_BATCH; b++) {
                k_lv_decide<<<lv_grid(bmax, LV_NODES), LV_BS, 0, s>>>(
                    L, st, c, sig, tkey, tval, dest, win, mn, mc, kin, kout);
                k_lv_conflict<<<lv_grid(bmax, LV_NODES), LV_BS, 0, s>>>(
                    L, st, c, sig, tkey, tval, dest, win, mn, mc, kin, kout);
                k_lv_apply<<<lv_grid(bmax, LV_BS), LV_BS, 0, s>>>(L, st, dest, c, sig, mn, mc,
                                                                  kin, kout, mv);
                k_lv_advance<<<1, 1, 0, s>>>(n, st);
            }
            read_scalars(W, W.counters, 5, s);
            const LvState *h = (const LvState *)(W.h_scal + 2);
            if (h->err) throw SlmError{4, "Louvain chunk made no progress"};
            if (h->p >= n) break;
        }
        const i64 moved = W.h_scal[0];
        if (moved == 0) {
            *converged = 1;
            break;
        }
        *moves += moved;
        passes++;
    }
    return passes;
}
