// The synchronous move sweep of MAXIMAL (Sec. 3.4): for every node i at once,
// w(i,C) for each neighbouring community C, join(i,C) = M2 w(i,C) - k_i S_C,
// the best C != c_i (key desc, label asc), and a move when it beats
// stay(i) = M2 w(i, c_i \ i) - k_i (S_ci - k_i).
//
// Rows are handled by lane groups sized to their degree class:
//   deg <= 32      4 or 8 lanes per row, every entry in registers; equal
//                  labels are found by shuffles (k_sweep_reg);
//   deg <= 512     32- or 64-lane groups with an LDS open-addressing table
//                  and a list of the occupied slots, so reading and clearing
//                  the table costs the number of distinct labels; groups loop
//                  over the rows of their bin with three rows in flight
//                  (k_sweep_pipe);
//   deg <= 4096    one 128- to 512-lane workgroup per row, same table
//                  (k_sweep_hash);
//   larger (hubs)  rows cut in HUB_CHUNK-entry chunks; a workgroup totals its
//                  chunk in LDS and writes its distinct labels grouped by a
//                  hash partition of the label space; one workgroup per
//                  (hub, partition) then totals them in LDS (no HBM atomics).
// A row starts from its descriptor (node, degree, first entry) in bin order;
// the short and pipelined rows gather a neighbour's (label, community total)
// in one 8-byte load.  The own community's weight never enters a table: it
// is summed in registers.  The bins are independent and may run on several
// streams at once.
#include "slm_forest.h"

// Home slot of label c in a table of H slots: the top bits of its hash for a
// power of two, else the hash scaled to [0, H) (multiply and keep the high
// word), so that a table can be 1.5x its bin's largest row.
template <int H> __device__ __forceinline__ u32 sw_slot(i32 c)
{
    if constexpr ((H & (H - 1)) == 0) {
        constexpr int LOG2H = __builtin_ctz(H);
        return hash_label(c) >> (32 - LOG2H);
    } else {
        return (u32)(((u64)hash_label(c) * (u64)H) >> 32);
    }
}

template <int H> __device__ __forceinline__ u32 sw_next(u32 h)
{
    if constexpr ((H & (H - 1)) == 0) return (h + 1) & (H - 1);
    else return h + 1 == (u32)H ? 0u : h + 1;
}

template <int G> __device__ __forceinline__ void sw_sync()
{
    if constexpr (G <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

__device__ __forceinline__ void write_move(const LevelView &L, i32 node, i32 ci, i64 ki, i64 win,
                                           i64 bk, i32 bc, const i32 *__restrict__ sigma,
                                           i32 *__restrict__ best_c, i64 *__restrict__ delta,
                                           i32 *__restrict__ w_own)
{
    const i64 yi = node_y(L, node);
    const i64 stay = node_m2(L, node) * win - ki * ((i64)sigma[ci] - ki) +
                     yi * (comm_y(L, ci) - yi);
    if (bc != INT32_MAX && bk > stay) {
        best_c[node] = bc;
        delta[node] = bk - stay;
    } else {
        best_c[node] = ci;
        delta[node] = 0;
    }
    w_own[node] = (i32)win;
}

// ------------------------------------------------------------------ isolated nodes
__global__ __launch_bounds__(SLM_BS) void k_sweep_zero(const i32 *__restrict__ nodes, i64 count,
                                                      const i32 *__restrict__ lab,
                                                      i32 *__restrict__ best_c,
                                                      i64 *__restrict__ delta,
                                                      i32 *__restrict__ w_own)
{
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < count;
         t += (i64)gridDim.x * blockDim.x) {
        const i32 u = nodes[t];
        best_c[u] = lab[u];
        delta[u] = 0;
        w_own[u] = 0;
    }
}

// ------------------------------------------------------------------ short rows
// ls[v] = (c_v, S_{c_v}): the short-row kernels gather a neighbour's label and
// its community's total in one load, so a row needs no second gather.
__global__ void k_pack_ls(const i32 *__restrict__ lab, const i32 *__restrict__ sigma, i64 n,
                          int2 *__restrict__ ls)
{
    for (i64 v = (i64)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (i64)gridDim.x * blockDim.x) {
        const i32 c = lab[v];
        ls[v] = make_int2(c, sigma[c]);
    }
}

// Rows of at most G*U entries: G lanes per row, U entries per lane, all in
// registers.  A row needs three dependent loads (its descriptor, its entries
// with its own (label, total), the neighbours' (label, total)); equal labels
// are found by comparing every entry of the group with every other through
// shuffles, and the first entry of each label (in row order) evaluates it.
template <int G, int U>
__global__ __launch_bounds__(SLM_BS) void k_sweep_reg(LevelView L, const int4 *__restrict__ rowd,
                                                     i64 count, const int2 *__restrict__ ls,
                                                     i32 *__restrict__ best_c,
                                                     i64 *__restrict__ delta,
                                                     i32 *__restrict__ w_own)
{
    constexpr int NG = SLM_BS / G;
    const int gl = threadIdx.x % G;
    const i64 slot = (i64)blockIdx.x * NG + threadIdx.x / G;
    const bool valid = slot < count;
    const int4 rd = valid ? rowd[slot] : make_int4(0, 0, 0, 0);
    const i32 node = rd.x;
    const int deg = rd.y;
    const i64 e0 = (i64)(u32)rd.z | ((i64)rd.w << 32);
    int2 ed[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int j = gl + u * G;
        ed[u] = (valid && j < deg) ? L.e[e0 + j] : make_int2(-1, 0);
    }
    const int2 own = valid ? ls[node] : make_int2(-1, 0);
    const i64 ki = valid ? L.k[node] : 0;
    const i64 m2 = valid ? node_m2(L, node) : 0;
    int2 lc[U];  // (label, total) of each entry's column; label -1: none
#pragma unroll
    for (int u = 0; u < U; u++)
        lc[u] = (ed[u].x >= 0 && ed[u].x != node) ? ls[ed[u].x] : make_int2(-1, 0);
    i64 win = 0;
    i64 tot[U];
    bool first[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        if (lc[u].x == own.x) win += ed[u].y;
        tot[u] = 0;
        first[u] = lc[u].x >= 0 && lc[u].x != own.x;
    }
#pragma unroll
    for (int v = 0; v < U; v++) {
        for (int j = 0; j < G; j++) {
            const i32 cj = __shfl(lc[v].x, j, G);
            const i32 wj = __shfl(ed[v].y, j, G);
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (cj == lc[u].x) {
                    tot[u] += wj;
                    if (v * G + j < u * G + gl) first[u] = false;
                }
            }
        }
    }
    i64 bk = INT64_MIN;
    i32 bc = INT32_MAX;
#pragma unroll
    for (int u = 0; u < U; u++) {
        if (!first[u]) continue;
        const i64 key = m2 * tot[u] - ki * (i64)lc[u].y + node_y(L, node) * comm_y(L, lc[u].x);
        if (better_key(key, lc[u].x, bk, bc)) {
            bk = key;
            bc = lc[u].x;
        }
    }
    win = group_sum<G, i64>(win);
    group_best<G>(bk, bc);
    if (valid && gl == 0) {
        const i64 yi = node_y(L, node);
        const i64 stay = m2 * win - ki * ((i64)own.y - ki) + yi * (comm_y(L, own.x) - yi);
        if (bc != INT32_MAX && bk > stay) {
            best_c[node] = bc;
            delta[node] = bk - stay;
        } else {
            best_c[node] = own.x;
            delta[node] = 0;
        }
        w_own[node] = (i32)win;
    }
}

// ------------------------------------------------------------------ LDS table with slot list
// One table per group; the groups of a workgroup loop over the nodes of the
// bin.  G lanes per node (G <= 64: the group lives in one wavefront; G > 64:
// the whole workgroup), H slots (H > max degree, about 1.5 to 2 times it), U = max degree / G
// entries per lane: a lane issues all its entry loads, then all its label
// gathers, before touching the table, so the memory latency of a row is paid
// about once.
// Adds w to label c in an LDS table of H slots (linear probing).  Returns the
// slot when c was new to the table, else -1.
template <int H>
__device__ __forceinline__ i32 table_add(i32 *keys, i32 *vals, i32 c, i32 w)
{
    u32 h = sw_slot<H>(c);
    for (int probe = 0; probe < H; probe++) {
        const i32 old = atomicCAS(&keys[h], -1, c);
        if (old == -1 || old == c) {
            atomicAdd(&vals[h], w);
            return old == -1 ? (i32)h : -1;
        }
        h = sw_next<H>(h);
    }
    return -1;
}

// Appends the slot s of every lane with s >= 0 to list[*cnt ..] (and x to
// xlist when X), one LDS atomic per group of G lanes in a wavefront instead
// of one per lane: the lanes of a group take consecutive places in lane
// order.  Groups of G >= 64 lanes may span several wavefronts sharing cnt.
template <int G, bool X>
__device__ __forceinline__ void group_append(i32 s, i32 *cnt, i32 *list, i32 *xlist, i32 x)
{
    const int lane = threadIdx.x & 63;
    const u64 bal = __ballot(s >= 0);
    u64 gm = ~0ull;
    if constexpr (G < 64) gm = (((u64)1 << G) - 1) << (lane & (64 - G));
    const u64 mine = bal & gm;
    const int rank = __popcll(mine & (((u64)1 << lane) - 1));
    const int leader = mine ? __ffsll((unsigned long long)mine) - 1 : lane;
    i32 base = 0;
    if (mine && lane == leader) base = atomicAdd(cnt, __popcll(mine));
    base = __shfl(base, leader, 64);
    if (s >= 0) {
        list[base + rank] = s;
        if constexpr (X) xlist[base + rank] = x;
    }
}

template <int G, int H, int U>
__global__ __launch_bounds__(G <= 64 ? SLM_BS : G) void k_sweep_hash(
    LevelView L, const i32 *__restrict__ nodes, i64 count, const i32 *__restrict__ lab,
    const i32 *__restrict__ sigma, i32 *__restrict__ best_c, i64 *__restrict__ delta,
    i32 *__restrict__ w_own)
{
    constexpr int NG = G <= 64 ? SLM_BS / G : 1;
    constexpr int BSZ = G <= 64 ? SLM_BS : G;
    constexpr int LIST = G * U;  // distinct labels of a row at most
    static_assert(H > LIST, "the table must exceed the longest row");
    __shared__ i32 s_key[NG * H];
    __shared__ i32 s_val[NG * H];
    __shared__ i32 s_list[NG * LIST];
    __shared__ i32 s_cnt[NG];
    __shared__ i64 red[32];
    const int gl = threadIdx.x % G, gi = threadIdx.x / G;
    i32 *keys = s_key + gi * H;
    i32 *vals = s_val + gi * H;
    i32 *list = s_list + gi * LIST;
    for (int i = threadIdx.x; i < NG * H; i += BSZ) {
        s_key[i] = -1;
        s_val[i] = 0;
    }
    if (threadIdx.x < NG) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    for (i64 slot = (i64)blockIdx.x * NG + gi; slot < count; slot += (i64)gridDim.x * NG) {
        const i32 node = nodes[slot];
        const i32 ci = lab[node];
        const i64 ki = L.k[node];
        const i64 m2 = node_m2(L, node);
        const i64 e0 = L.rp[node];
        const int deg = (int)(L.rp[node + 1] - e0);
        int2 ed[U];
        i32 c[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = gl + u * G;
            ed[u] = j < deg ? L.e[e0 + j] : make_int2(-1, 0);
        }
#pragma unroll
        for (int u = 0; u < U; u++) c[u] = (ed[u].x >= 0 && ed[u].x != node) ? lab[ed[u].x] : -1;
        i64 win = 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
            i32 sl = -1;
            if (c[u] >= 0) {
                if (c[u] == ci) win += ed[u].y;
                else sl = table_add<H>(keys, vals, c[u], ed[u].y);
            }
            group_append<G, false>(sl, &s_cnt[gi], list, nullptr, 0);
        }
        sw_sync<G>();
        const int nd = s_cnt[gi];
        i64 bk = INT64_MIN;
        i32 bc = INT32_MAX;
        for (int i = gl; i < nd; i += G) {
            const i32 h = list[i];
            const i32 cc = keys[h];
            const i64 key = m2 * (i64)vals[h] - ki * (i64)sigma[cc] +
                            node_y(L, node) * comm_y(L, cc);
            if (better_key(key, cc, bk, bc)) {
                bk = key;
                bc = cc;
            }
            keys[h] = -1;
            vals[h] = 0;
        }
        if constexpr (G <= 64) {
            win = group_sum<G, i64>(win);
            group_best<G>(bk, bc);
        } else {
            win = block_sum<i64>(win, red);
            block_best(bk, bc, red);
        }
        if (gl == 0) {
            write_move(L, node, ci, ki, win, bk, bc, sigma, best_c, delta, w_own);
            s_cnt[gi] = 0;
        }
        sw_sync<G>();
    }
}

// Pipelined rows of a bin for groups of at most 64 lanes.  A row's loads form
// a chain (descriptor -> entries -> neighbours' (label, total)); the loop
// keeps three rows in flight: while row i is inserted into the table, the
// entries of row i+1 and the descriptor of row i+2 are loading, and while
// row i's table is read, row i+1's labels are.  The community total of each
// table entry comes with its label (ls) and is kept beside the slot list, so
// the table's read-out needs no further load.
template <int G, int H, int U>
__global__ __launch_bounds__(SLM_BS) void k_sweep_pipe(LevelView L, const int4 *__restrict__ rowd,
                                                      i64 count, const int2 *__restrict__ ls,
                                                      i32 *__restrict__ best_c,
                                                      i64 *__restrict__ delta,
                                                      i32 *__restrict__ w_own)
{
    static_assert(G <= 64, "one wavefront per group at most");
    constexpr int NG = SLM_BS / G;
    constexpr int LIST = G * U;  // distinct labels of a row at most
    static_assert(H > LIST, "the table must exceed the longest row");
    __shared__ i32 s_key[NG * H];
    __shared__ i32 s_val[NG * H];
    __shared__ i32 s_list[NG * LIST];
    __shared__ i32 s_lsig[NG * LIST];
    __shared__ i32 s_cnt[NG];
    const int gl = threadIdx.x % G, gi = threadIdx.x / G;
    i32 *keys = s_key + gi * H;
    i32 *vals = s_val + gi * H;
    i32 *list = s_list + gi * LIST;
    i32 *lsig = s_lsig + gi * LIST;
    for (int i = threadIdx.x; i < NG * H; i += SLM_BS) {
        s_key[i] = -1;
        s_val[i] = 0;
    }
    if (threadIdx.x < NG) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    const i64 stride = (i64)gridDim.x * NG;
    i64 slot = (i64)blockIdx.x * NG + gi;
    // row i (current), row i+1 (next: descriptor and entries), row i+2 (descriptor)
    int4 rd = slot < count ? rowd[slot] : make_int4(-1, 0, 0, 0);
    int4 rd1 = slot + stride < count ? rowd[slot + stride] : make_int4(-1, 0, 0, 0);
    int2 ed[U], lc[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int j = gl + u * G;
        ed[u] = (rd.x >= 0 && j < rd.y)
                    ? L.e[((i64)(u32)rd.z | ((i64)rd.w << 32)) + j]
                    : make_int2(-1, 0);
    }
#pragma unroll
    for (int u = 0; u < U; u++)
        lc[u] = (ed[u].x >= 0 && ed[u].x != rd.x) ? ls[ed[u].x] : make_int2(-1, 0);
    int2 own = rd.x >= 0 ? ls[rd.x] : make_int2(-1, 0);
    i64 ki = rd.x >= 0 ? (i64)L.k[rd.x] : 0;
    i64 m2 = rd.x >= 0 ? node_m2(L, rd.x) : 0;
    while (slot < count) {
        // next rows' loads: entries of i+1, descriptor of i+2
        const i64 s2 = slot + 2 * stride;
        const int4 rd2 = s2 < count ? rowd[s2] : make_int4(-1, 0, 0, 0);
        int2 ed1[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int j = gl + u * G;
            ed1[u] = (rd1.x >= 0 && j < rd1.y)
                         ? L.e[((i64)(u32)rd1.z | ((i64)rd1.w << 32)) + j]
                         : make_int2(-1, 0);
        }
        // row i into the table
        i64 win = 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const i32 c = lc[u].x;
            i32 sl = -1;
            if (c >= 0) {
                if (c == own.x) win += ed[u].y;
                else sl = table_add<H>(keys, vals, c, ed[u].y);
            }
            group_append<G, true>(sl, &s_cnt[gi], list, lsig, lc[u].y);
        }
        sw_sync<G>();
        // labels of row i+1 while row i's table is read
        int2 lc1[U];
#pragma unroll
        for (int u = 0; u < U; u++)
            lc1[u] = (ed1[u].x >= 0 && ed1[u].x != rd1.x) ? ls[ed1[u].x] : make_int2(-1, 0);
        const int2 own1 = rd1.x >= 0 ? ls[rd1.x] : make_int2(-1, 0);
        const i64 ki1 = rd1.x >= 0 ? (i64)L.k[rd1.x] : 0;
        const i64 m21 = rd1.x >= 0 ? node_m2(L, rd1.x) : 0;
        const int nd = s_cnt[gi];
        i64 bk = INT64_MIN;
        i32 bc = INT32_MAX;
        for (int i = gl; i < nd; i += G) {
            const i32 h = list[i];
            const i32 cc = keys[h];
            const i64 key = m2 * (i64)vals[h] - ki * (i64)lsig[i] + node_y(L, rd.x) * comm_y(L, cc);
            if (better_key(key, cc, bk, bc)) {
                bk = key;
                bc = cc;
            }
            keys[h] = -1;
            vals[h] = 0;
        }
        win = group_sum<G, i64>(win);
        group_best<G>(bk, bc);
        if (gl == 0) {
            const i32 node = rd.x;
            const i64 yi = node_y(L, node);
            const i64 stay = m2 * win - ki * ((i64)own.y - ki) + yi * (comm_y(L, own.x) - yi);
            if (bc != INT32_MAX && bk > stay) {
                best_c[node] = bc;
                delta[node] = bk - stay;
            } else {
                best_c[node] = own.x;
                delta[node] = 0;
            }
            w_own[node] = (i32)win;
            s_cnt[gi] = 0;
        }
        sw_sync<G>();
        // advance
        slot += stride;
        rd = rd1;
        rd1 = rd2;
#pragma unroll
        for (int u = 0; u < U; u++) {
            ed[u] = ed1[u];
            lc[u] = lc1[u];
        }
        own = own1;
        ki = ki1;
        m2 = m21;
    }
}

// ------------------------------------------------------------------ hub rows
// A hub row is cut in HUB_CHUNK-entry chunks.  A chunk totals its entries by
// label in LDS, then writes its distinct (label, weight) pairs grouped by a
// partition of the label space (the top bits of a second hash, P_h = 2^logp
// partitions per hub, about HUB_PART labels each): poff gives, for every
// partition, where the chunk's group starts.  One workgroup per (hub,
// partition) then totals the groups of all the hub's chunks in LDS and keeps
// its best label.  No step needs an atomic on HBM.
#define HUB_H 4096      // LDS slots of a chunk table
#define HUB_BS 256

__device__ __forceinline__ u32 hub_part_hash(i32 c)
{
    return (u32)c * 0x85EBCA77u;  // odd: a bijection of the 32-bit labels
}

// Exclusive prefix sum over the 256 threads of a workgroup; *total gets the
// sum.  wsum: 4 slots of LDS.
__device__ __forceinline__ i32 block_excl_scan(i32 v, i32 *wsum, i32 *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    i32 x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const i32 y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    __syncthreads();
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    i32 off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SLM_BS / 64; w++) {
        if (w < wid) off += wsum[w];
        tot += wsum[w];
    }
    *total = tot;
    return off + x - v;
}

__global__ __launch_bounds__(HUB_BS) void k_sweep_hub_chunk(
    LevelView L, const HubChunk *__restrict__ hchunk, const i32 *__restrict__ lab,
    int2 *__restrict__ part, i64 *__restrict__ poff, i32 *__restrict__ cwin)
{
    __shared__ i32 keys[HUB_H];
    __shared__ i32 vals[HUB_H];
    __shared__ i32 list[HUB_CHUNK];
    __shared__ i32 hist[HUB_PMAX];
    __shared__ int cnt;
    __shared__ i32 wsum[SLM_BS / 64];
    __shared__ i64 red[32];
    const HubChunk hc = hchunk[blockIdx.x];
    const int logp = hc.logp;
    const int P = 1 << logp;
    for (int i = threadIdx.x; i < HUB_H; i += HUB_BS) {
        keys[i] = -1;
        vals[i] = 0;
    }
    for (int i = threadIdx.x; i < P; i += HUB_BS) hist[i] = 0;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const i32 node = hc.node;
    const i32 ci = lab[node];
    const i64 b = hc.beg, end = hc.end;
    constexpr int U = HUB_CHUNK / HUB_BS;
    int2 ed[U];
    i32 c[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const i64 j = b + threadIdx.x + (i64)u * HUB_BS;
        ed[u] = j < end ? L.e[j] : make_int2(-1, 0);
    }
#pragma unroll
    for (int u = 0; u < U; u++) c[u] = (ed[u].x >= 0 && ed[u].x != node) ? lab[ed[u].x] : -1;
    i64 win = 0;
#pragma unroll
    for (int u = 0; u < U; u++) {
        i32 sl = -1;
        if (c[u] >= 0) {
            if (c[u] == ci) win += ed[u].y;
            else sl = table_add<HUB_H>(keys, vals, c[u], ed[u].y);
        }
        group_append<64, false>(sl, &cnt, list, nullptr, 0);
    }
    __syncthreads();
    // partition of each distinct label, and its rank inside the partition
    const int nd = cnt;
    int pr[U], rk[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int i = threadIdx.x + u * HUB_BS;
        pr[u] = -1;
        if (i < nd) {
            const i32 cc = keys[list[i]];
            pr[u] = logp ? (int)(hub_part_hash(cc) >> (32 - logp)) : 0;
            rk[u] = atomicAdd(&hist[pr[u]], 1);
        }
    }
    __syncthreads();
    // exclusive prefix of the partition counts (P <= 4 * HUB_BS)
    constexpr int PT = HUB_PMAX / HUB_BS;
    i32 loc[PT];
    i32 mine = 0;
#pragma unroll
    for (int q = 0; q < PT; q++) {
        const int p = threadIdx.x * PT + q;
        loc[q] = p < P ? hist[p] : 0;
        mine += loc[q];
    }
    i32 tot;
    i32 run = block_excl_scan(mine, wsum, &tot);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PT; q++) {
        const int p = threadIdx.x * PT + q;
        if (p < P) hist[p] = run;
        run += loc[q];
    }
    __syncthreads();
    const i64 ob = hc.out;
    const i64 pb = hc.pbase;
    for (int p = threadIdx.x; p <= P; p += HUB_BS) poff[pb + p] = ob + (p < P ? hist[p] : nd);
#pragma unroll
    for (int u = 0; u < U; u++) {
        if (pr[u] < 0) continue;
        const i32 s = list[threadIdx.x + u * HUB_BS];
        part[ob + hist[pr[u]] + rk[u]] = make_int2(keys[s], vals[s]);
    }
    win = block_sum<i64>(win, red);
    if (threadIdx.x == 0) cwin[blockIdx.x] = (i32)win;
}

// Adds w to label c in an LDS table of 2^tbits slots (tbits <= log2 HUB_TH);
// false if the table is full (then nothing changes).
__device__ __forceinline__ bool tile_insert(i32 *keys, i32 *vals, int tbits, i32 c, i32 w)
{
    const u32 mask = (1u << tbits) - 1;
    u32 h = hash_label(c) >> (32 - tbits);
    for (u32 probe = 0; probe <= mask; probe++) {
        const i32 old = atomicCAS(&keys[h], -1, c);
        if (old == -1 || old == c) {
            atomicAdd(&vals[h], w);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

// Best label of one partition of one hub: the pairs of every chunk of the
// hub that fall in the partition are totalled in an LDS table of 2^tbits
// slots, then keyed.  A partition holding more than cap pairs is taken in
// 2^logs passes, each over the labels whose next logs hash bits equal the
// pass number.  As the hash is a bijection, a pass can see at most
// 2^(32-logp-logs) distinct labels, so doubling the passes after a pass
// filled the table ends with every pass fitting.
__global__ __launch_bounds__(SLM_BS) void k_sweep_hub_tile(
    LevelView L, const HubTile *__restrict__ htile, const int2 *__restrict__ part,
    const i64 *__restrict__ poff, const i32 *__restrict__ sigma, int cap, int tbits,
    i64 *__restrict__ tile_key, i32 *__restrict__ tile_id)
{
    __shared__ i32 keys[HUB_TH];
    __shared__ i32 vals[HUB_TH];
    __shared__ i64 segb[SLM_BS];
    __shared__ i32 pre[SLM_BS];
    __shared__ i32 wsum[SLM_BS / 64];
    __shared__ int full;
    __shared__ i64 red[32];
    const HubTile ht = htile[blockIdx.x];
    const int p = ht.p;
    const int logp = ht.logp;
    const i64 pstride = ((i64)1 << logp) + 1;  // offsets per chunk
    const i64 pb0 = ht.pbase0 + p;              // this partition's offset in chunk 0
    const i32 c0 = 0, c1 = ht.nch;              // chunks, numbered within the hub
    const i32 node = ht.node;
    const i64 ki = L.k[node];
    const i64 m2 = node_m2(L, node);
    // pairs in this partition over all chunks
    i64 tot = 0;
    for (i32 ch = c0 + threadIdx.x; ch < c1; ch += SLM_BS) {
        const i64 pb = pb0 + ch * pstride;
        tot += poff[pb + 1] - poff[pb];
    }
    tot = block_sum<i64>(tot, red);
    int logs = 0;
    while (((i64)cap << logs) < tot && logp + logs < 32) logs++;
    i64 bk = INT64_MIN;
    i32 bc = INT32_MAX;
    for (;;) {
        bool failed = false;
        for (int q = 0; q < (1 << logs) && !failed; q++) {
            for (int i = threadIdx.x; i < (1 << tbits); i += SLM_BS) {
                keys[i] = -1;
                vals[i] = 0;
            }
            if (threadIdx.x == 0) full = 0;
            for (i32 cb = c0; cb < c1; cb += SLM_BS) {
                const i32 ch = cb + threadIdx.x;
                i64 lo = 0, hi = 0;
                if (ch < c1) {
                    const i64 pb = pb0 + ch * pstride;
                    lo = poff[pb];
                    hi = poff[pb + 1];
                }
                i32 n_all;
                const i32 ex = block_excl_scan((i32)(hi - lo), wsum, &n_all);
                segb[threadIdx.x] = lo;
                pre[threadIdx.x] = ex;
                __syncthreads();
                const int nb = c1 - cb < SLM_BS ? c1 - cb : SLM_BS;
                for (i32 j = threadIdx.x; j < n_all; j += SLM_BS) {
                    int k0 = 0, k1 = nb;  // last k with pre[k] <= j
                    while (k1 - k0 > 1) {
                        const int mid = (k0 + k1) >> 1;
                        if (pre[mid] <= j) k0 = mid;
                        else k1 = mid;
                    }
                    const int2 cv = part[segb[k0] + (j - pre[k0])];
                    if (logs > 0 &&
                        (int)((hub_part_hash(cv.x) << logp) >> (32 - logs)) != q)
                        continue;
                    if (!tile_insert(keys, vals, tbits, cv.x, cv.y)) full = 1;
                }
                __syncthreads();
            }
            failed = full != 0;
            __syncthreads();  // every thread has read full before it is reset
            if (failed) break;
            for (int i = threadIdx.x; i < (1 << tbits); i += SLM_BS) {
                const i32 cc = keys[i];
                if (cc >= 0) {
                    const i64 key = m2 * (i64)vals[i] - ki * (i64)sigma[cc] +
                                    node_y(L, node) * comm_y(L, cc);
                    if (better_key(key, cc, bk, bc)) {
                        bk = key;
                        bc = cc;
                    }
                }
            }
            __syncthreads();
        }
        if (!failed) break;
        logs++;
        bk = INT64_MIN;
        bc = INT32_MAX;
    }
    block_best(bk, bc, red);
    if (threadIdx.x == 0) {
        tile_key[blockIdx.x] = bk;
        tile_id[blockIdx.x] = bc;
    }
}

__global__ __launch_bounds__(64) void k_sweep_hub_final(
    LevelView L, const i32 *__restrict__ hub_node, const i32 *__restrict__ tile_first,
    const i32 *__restrict__ chunk_first, const i32 *__restrict__ lab,
    const i32 *__restrict__ sigma, const i64 *__restrict__ tile_key,
    const i32 *__restrict__ tile_id, const i32 *__restrict__ cwin, i32 *__restrict__ best_c,
    i64 *__restrict__ delta, i32 *__restrict__ w_own)
{
    const i32 h = blockIdx.x;
    i64 bk = INT64_MIN;
    i32 bc = INT32_MAX;
    for (i32 t = tile_first[h] + threadIdx.x; t < tile_first[h + 1]; t += 64)
        if (better_key(tile_key[t], tile_id[t], bk, bc)) {
            bk = tile_key[t];
            bc = tile_id[t];
        }
    group_best<64>(bk, bc);
    i64 win = 0;
    for (i32 ch = chunk_first[h] + threadIdx.x; ch < chunk_first[h + 1]; ch += 64) win += cwin[ch];
    win = group_sum<64>(win);
    if (threadIdx.x == 0) {
        const i32 node = hub_node[h];
        write_move(L, node, lab[node], L.k[node], win, bk, bc, sigma, best_c, delta, w_own);
    }
}

// ------------------------------------------------------------------ dispatch
static unsigned persistent_grid(i64 count, int per_block, int max_blocks)
{
    i64 g = (count + per_block - 1) / per_block;
    if (g > max_blocks) g = max_blocks;
    if (g < 1) g = 1;
    return (unsigned)g;
}

static int grid_of(const Bins &Bn, int b)
{
    return Bn.grid_cap[b] > 0 ? Bn.grid_cap[b] : 8192;
}

void run_sweep(const LevelView &L, const Bins &Bn, const i32 *lab, const i32 *sigma,
               i32 *best_c, i64 *delta, i32 *w_own, int2 *hub_part, i64 *hub_poff,
               i32 *hub_cwin, i64 *hub_tile_key, i32 *hub_tile_id, hipStream_t s,
               const Fanout *F)
{
    // streams: the hub chain and the zero rows stay on s; the other bins go
    // to the side streams, longest first
    hipStream_t st[FAN_SIDE];
    for (int q = 0; q < FAN_SIDE; q++) st[q] = F ? F->side[q] : s;
    if (L.n > 0) {
        i64 gp = (L.n + SLM_BS - 1) / SLM_BS;
        if (gp > 16384) gp = 16384;
        k_pack_ls<<<(unsigned)gp, SLM_BS, 0, s>>>(lab, sigma, L.n, Bn.ls);
    }
    if (F) {
        HIPCHK(hipEventRecord(F->fork, s));
        for (int q = 0; q < FAN_SIDE; q++) HIPCHK(hipStreamWaitEvent(F->side[q], F->fork, 0));
    }
    const i32 *nodes;
    i64 cnt;
#define HASH_BIN(B, G, H, U, STREAM)                                                   \
    cnt = Bn.off[B + 1] - Bn.off[B];                                                   \
    nodes = Bn.nodes + Bn.off[B];                                                      \
    if (cnt > 0)                                                                       \
        k_sweep_hash<G, H, U>                                                          \
            <<<persistent_grid(cnt, G <= 64 ? SLM_BS / G : 1, grid_of(Bn, B)),               \
               G <= 64 ? SLM_BS : G,                                                   \
               0, STREAM>>>(L, nodes, cnt, lab, sigma, best_c, delta, w_own);
#define PIPE_BIN(B, G, H, U, STREAM)                                                   \
    cnt = Bn.off[B + 1] - Bn.off[B];                                                   \
    if (cnt > 0)                                                                       \
        k_sweep_pipe<G, H, U><<<persistent_grid(cnt, SLM_BS / G, grid_of(Bn, B)), SLM_BS, 0,  \
                                STREAM>>>(                                             \
            L, Bn.rowd + Bn.off[B], cnt, Bn.ls, best_c, delta, w_own);
    PIPE_BIN(BIN_512, 64, 752, 8, st[0])
    PIPE_BIN(BIN_256, 64, 512, 4, st[0])
    PIPE_BIN(BIN_128, 64, 256, 2, st[1])
    PIPE_BIN(BIN_64, 32, 128, 2, st[1])
    HASH_BIN(BIN_2048, 256, 3008, 8, st[2])
    HASH_BIN(BIN_1024, 128, 2048, 8, st[2])
    HASH_BIN(BIN_4096, 512, 6144, 8, st[2])
#undef HASH_BIN
#undef PIPE_BIN
    cnt = Bn.off[BIN_32 + 1] - Bn.off[BIN_32];
    if (cnt > 0)
        k_sweep_reg<8, 4><<<grid_for(cnt, SLM_BS / 8), SLM_BS, 0, st[1]>>>(
            L, Bn.rowd + Bn.off[BIN_32], cnt, Bn.ls, best_c, delta, w_own);
    cnt = Bn.off[BIN_8 + 1] - Bn.off[BIN_8];
    if (cnt > 0)
        k_sweep_reg<4, 2><<<grid_for(cnt, SLM_BS / 4), SLM_BS, 0, st[2]>>>(
            L, Bn.rowd + Bn.off[BIN_8], cnt, Bn.ls, best_c, delta, w_own);
    if (Bn.nhub > 0) {
        k_sweep_hub_chunk<<<(unsigned)Bn.nchunk, HUB_BS, 0, s>>>(L, Bn.hchunk, lab, hub_part,
                                                                hub_poff, hub_cwin);
        k_sweep_hub_tile<<<(unsigned)Bn.ntile, SLM_BS, 0, s>>>(L, Bn.htile, hub_part, hub_poff,
                                                              sigma, Bn.hub_cap, Bn.hub_tbits,
                                                              hub_tile_key, hub_tile_id);
        k_sweep_hub_final<<<(unsigned)Bn.nhub, 64, 0, s>>>(
            L, Bn.hub_node, Bn.tile_off_of_hub, Bn.chunk_off_of_hub, lab, sigma, hub_tile_key,
            hub_tile_id, hub_cwin, best_c, delta, w_own);
    }
    cnt = Bn.off[BIN_ZERO + 1] - Bn.off[BIN_ZERO];
    nodes = Bn.nodes + Bn.off[BIN_ZERO];
    if (cnt > 0)
        k_sweep_zero<<<persistent_grid(cnt, SLM_BS, 2048), SLM_BS, 0, s>>>(nodes, cnt, lab, best_c,
                                                                          delta, w_own);
    if (F) {
        for (int q = 0; q < FAN_SIDE; q++) {
            HIPCHK(hipEventRecord(F->join[q], F->side[q]));
            HIPCHK(hipStreamWaitEvent(s, F->join[q], 0));
        }
    }
}
