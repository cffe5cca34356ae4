// Row kernels: every node's CSR row is handled by a group of lanes sized to
// its degree (the degree bins of slm_impl.h).  Groups of up to 64 lanes live
// inside one wavefront and keep their per-node community table in LDS; the
// 2048- and 4096-entry bins use a whole workgroup per node; hub rows are cut
// in HUB_CHUNK-entry chunks spread over workgroups with the table in HBM.
//
// Kernels here: strengths (Sec. 2.4), ASSIGN (Sec. 3.1), the MAXIMAL sweep
// and re-pointing (Sec. 3.4), own-community weights, and the per-row
// pre-aggregation of AGGREGATE (Sec. 3.5).
#include "slm_forest.h"

// Group shapes per bin: lanes per node G and LDS table slots H (>= 2*deg).
template <int B> struct BinShape;
template <> struct BinShape<BIN_ZERO> { static constexpr int G = 1, H = 2; };
template <> struct BinShape<BIN_8> { static constexpr int G = 8, H = 16; };
template <> struct BinShape<BIN_32> { static constexpr int G = 32, H = 64; };
template <> struct BinShape<BIN_64> { static constexpr int G = 32, H = 128; };
template <> struct BinShape<BIN_128> { static constexpr int G = 64, H = 256; };
template <> struct BinShape<BIN_256> { static constexpr int G = 64, H = 512; };
template <> struct BinShape<BIN_512> { static constexpr int G = 64, H = 1024; };
template <> struct BinShape<BIN_1024> { static constexpr int G = 128, H = 2048; };
template <> struct BinShape<BIN_2048> { static constexpr int G = 256, H = 4096; };
template <> struct BinShape<BIN_4096> { static constexpr int G = 512, H = 8192; };

template <int G> struct GroupGeom {
    static constexpr int NG = (G <= 64) ? SLM_BS / G : 1;  // groups per workgroup
    static constexpr int BSZ = (G <= 64) ? SLM_BS : G;     // workgroup size
};

template <int H> __device__ __forceinline__ u32 slot_of(i32 c)
{
    constexpr int LOG2H = __builtin_ctz(H);
    return LOG2H == 0 ? 0u : (hash_label(c) >> (32 - LOG2H));
}

// Orders LDS accesses of the lanes of one group.
template <int G> __device__ __forceinline__ void group_sync()
{
    if constexpr (G <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

template <int G, typename T> __device__ __forceinline__ T gsum(T v, i64 *red)
{
    if constexpr (G == 1) return v;
    else if constexpr (G <= 64) return group_sum<G, T>(v);
    else return block_sum<T>(v, red);
}

template <int G> __device__ __forceinline__ void gbest(i64 &k, i32 &id, i64 *red)
{
    if constexpr (G == 1) return;
    else if constexpr (G <= 64) group_best<G>(k, id);
    else block_best(k, id, red);
}

// Exclusive scan of one int per lane over the group; *total = group sum.
template <int G> __device__ __forceinline__ int gscan(int v, int &total, i64 *red)
{
    if constexpr (G == 1) {
        total = v;
        return 0;
    } else if constexpr (G <= 64) {
        const int gl = threadIdx.x & (G - 1);
        int inc = v;
#pragma unroll
        for (int d = 1; d < G; d <<= 1) {
            int t = __shfl_up(inc, d, G);
            if (gl >= d) inc += t;
        }
        total = __shfl(inc, G - 1, G);
        return inc - v;
    } else {
        const int lane = threadIdx.x & 63, wid = threadIdx.x / 64, nw = blockDim.x / 64;
        int inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        __syncthreads();
        if (lane == 63) red[wid] = inc;
        __syncthreads();
        int before = 0, tot = 0;
        for (int w = 0; w < nw; w++) {
            if (w < wid) before += (int)red[w];
            tot += (int)red[w];
        }
        __syncthreads();
        total = tot;
        return before + inc - v;
    }
}

#define GROUP_PROLOGUE(G)                                                            \
    constexpr int NG = GroupGeom<G>::NG;                                             \
    const int gl = (int)(threadIdx.x % (G));                                         \
    const int gi = (int)(threadIdx.x / (G));                                         \
    const i64 slot = (i64)blockIdx.x * NG + gi;                                      \
    const bool valid = slot < count;                                                 \
    const i32 node = valid ? nodes[slot] : 0;

// ------------------------------------------------------------------ strengths
template <int G>
__global__ __launch_bounds__(GroupGeom<G>::BSZ) void k_strength(
    const i64 *__restrict__ rp, const int2 *__restrict__ e, const i32 *__restrict__ nodes,
    i64 count, i32 *__restrict__ k, i32 *__restrict__ diag)
{
    __shared__ i64 red[32];
    GROUP_PROLOGUE(G)
    i64 s = 0, d = 0;
    if (valid) {
        for (i64 j = rp[node] + gl; j < rp[node + 1]; j += G) {
            int2 ed = e[j];
            s += ed.y;
            if (ed.x == node) d += ed.y;
        }
    }
    s = gsum<G>(s, red);
    d = gsum<G>(d, red);
    if (valid && gl == 0) {
        k[node] = (i32)s;
        diag[node] = (i32)d;
    }
}

// *acc += sum of k[0..n): a bounded grid, one atomic per workgroup.
__global__ __launch_bounds__(SLM_BS) void k_sum_i32(const i32 *__restrict__ k, i64 n,
                                                   i64 *__restrict__ acc)
{
    __shared__ i64 red[SLM_BS / 64];
    i64 t = 0;
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (i64)gridDim.x * blockDim.x)
        t += k[i];
    t = block_sum<i64>(t, red);
    if (threadIdx.x == 0 && t) atomicAdd((unsigned long long *)acc, (unsigned long long)t);
}

// ------------------------------------------------------------------ ASSIGN / re-point
// ASSIGN keeps the best neighbour if its pair key is positive, else the node
// itself.  Re-pointing takes the best neighbour in the target community; an
// accepted node always has one (its target is a neighbour's label), so
// finding none means the inputs disagree: the node keeps its pointer and
// err is raised instead of writing an id that is no node.
template <bool REPOINT>
__device__ __forceinline__ void write_assign(i32 *a, i32 node, i64 bk, i32 bj, int *err)
{
    if (REPOINT) {
        if (bj != INT32_MAX) a[node] = bj;
        else if (err) *err = 1;
    } else {
        a[node] = (bj != INT32_MAX && bk > 0) ? bj : node;
    }
}

// REPOINT = false: a[i] = argmax_{j != i} pair(i,j) if positive, else i.
// REPOINT = true : for accepted i, a[i] = argmax_{j: lab j = best_c i} pair(i,j).
template <int G, bool REPOINT>
__global__ __launch_bounds__(GroupGeom<G>::BSZ) void k_argmax(
    LevelView L, const i32 *__restrict__ nodes, i64 count, const i32 *__restrict__ lab,
    const i32 *__restrict__ best_c, const uint8_t *__restrict__ accept, i32 *__restrict__ a,
    int *__restrict__ err)
{
    __shared__ i64 red[32];
    GROUP_PROLOGUE(G)
    bool active = valid;
    if constexpr (REPOINT) active = valid && accept[node];
    i64 bk = INT64_MIN;
    i32 bj = INT32_MAX;
    if (active) {
        const i64 ki = L.k[node];
        const i64 yi = node_y(L, node);
        const i64 m2 = node_m2(L, node);
        const i32 D = REPOINT ? best_c[node] : 0;
        for (i64 j = L.rp[node] + gl; j < L.rp[node + 1]; j += G) {
            int2 ed = L.e[j];
            const i32 v = ed.x;
            if (v == node) continue;
            if (REPOINT && lab[v] != D) continue;
            i64 key = m2 * (i64)ed.y - ki * (i64)L.k[v] + yi * node_y(L, v);
            if (better_key(key, v, bk, bj)) {
                bk = key;
                bj = v;
            }
        }
    }
    gbest<G>(bk, bj, red);
    if (active && gl == 0) write_assign<REPOINT>(a, node, bk, bj, err);
}

// ------------------------------------------------------------------ own-community weight
template <int G>
__global__ __launch_bounds__(GroupGeom<G>::BSZ) void k_own(
    LevelView L, const i32 *__restrict__ nodes, i64 count, const i32 *__restrict__ lab,
    const uint8_t *__restrict__ active, i32 *__restrict__ wc)
{
    __shared__ i64 red[32];
    GROUP_PROLOGUE(G)
    const i32 ci = valid ? lab[node] : 0;
    const bool act = valid && (active == nullptr || active[ci]);
    i64 s = 0;
    if (act) {
        for (i64 j = L.rp[node] + gl; j < L.rp[node + 1]; j += G) {
            int2 ed = L.e[j];
            if (lab[ed.x] == ci) s += ed.y;
        }
    }
    s = gsum<G>(s, red);
    if (act && gl == 0) wc[node] = (i32)s;
}

// ------------------------------------------------------------------ short rows in registers
// Rows of at most G*U entries (degree bins up to 64): G lanes per row, U
// entries per lane, loaded together from the row descriptor (node, degree,
// first entry), then every neighbour gathered together: two dependent loads
// per row instead of a loop.
template <int G, int U, bool REPOINT>
__global__ __launch_bounds__(SLM_BS) void k_argmax_reg(
    LevelView L, const int4 *__restrict__ rowd, i64 count, const i32 *__restrict__ lab,
    const i32 *__restrict__ best_c, const uint8_t *__restrict__ accept, i32 *__restrict__ a,
    int *__restrict__ err)
{
    constexpr int NG = SLM_BS / G;
    const int gl = threadIdx.x % G;
    const i64 slot = (i64)blockIdx.x * NG + threadIdx.x / G;
    const bool valid = slot < count;
    const int4 rd = valid ? rowd[slot] : make_int4(0, 0, 0, 0);
    const i32 node = rd.x;
    const i64 e0 = (i64)(u32)rd.z | ((i64)rd.w << 32);
    bool active = valid;
    if constexpr (REPOINT) active = valid && accept[node];
    int2 ed[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int j = gl + u * G;
        ed[u] = (active && j < rd.y) ? L.e[e0 + j] : make_int2(-1, 0);
    }
    const i64 ki = active ? (i64)L.k[node] : 0;
    const i64 yi = active ? node_y(L, node) : 0;
    const i64 m2 = active ? node_m2(L, node) : 0;
    const i32 D = (REPOINT && active) ? best_c[node] : 0;
    i32 kv[U], lv[U], yv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const i32 v = ed[u].x;
        const bool ok = v >= 0 && v != node;
        kv[u] = ok ? L.k[v] : 0;
        lv[u] = (REPOINT && ok) ? lab[v] : 0;
        yv[u] = ok ? (i32)node_y(L, v) : 0;
    }
    i64 bk = INT64_MIN;
    i32 bj = INT32_MAX;
#pragma unroll
    for (int u = 0; u < U; u++) {
        const i32 v = ed[u].x;
        if (v < 0 || v == node) continue;
        if (REPOINT && lv[u] != D) continue;
        const i64 key = m2 * (i64)ed[u].y - ki * (i64)kv[u] + yi * (i64)yv[u];
        if (better_key(key, v, bk, bj)) {
            bk = key;
            bj = v;
        }
    }
    group_best<G>(bk, bj);
    if (active && gl == 0) write_assign<REPOINT>(a, node, bk, bj, err);
}

template <int G, int U>
__global__ __launch_bounds__(SLM_BS) void k_own_reg(
    LevelView L, const int4 *__restrict__ rowd, i64 count, const i32 *__restrict__ lab,
    const uint8_t *__restrict__ active, i32 *__restrict__ wc)
{
    constexpr int NG = SLM_BS / G;
    const int gl = threadIdx.x % G;
    const i64 slot = (i64)blockIdx.x * NG + threadIdx.x / G;
    const bool valid = slot < count;
    const int4 rd = valid ? rowd[slot] : make_int4(0, 0, 0, 0);
    const i32 node = rd.x;
    const i64 e0 = (i64)(u32)rd.z | ((i64)rd.w << 32);
    const i32 ci = valid ? lab[node] : 0;
    int2 ed[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int j = gl + u * G;
        ed[u] = (valid && j < rd.y) ? L.e[e0 + j] : make_int2(-1, 0);
    }
    const bool act = valid && (active == nullptr || active[ci]);
    i32 lv[U];
#pragma unroll
    for (int u = 0; u < U; u++) lv[u] = (act && ed[u].x >= 0) ? lab[ed[u].x] : -1;
    i64 s = 0;
#pragma unroll
    for (int u = 0; u < U; u++)
        if (lv[u] == ci && ed[u].x >= 0) s += ed[u].y;
    s = group_sum<G, i64>(s);
    if (act && gl == 0) wc[node] = (i32)s;
}

// ------------------------------------------------------------------ contraction rows
// Per row u: distinct (lab_u, lab_v) with summed weights (own community and
// diagonal included), written at rec[rp[u] ..]; cnt[u] = their number.
template <int G, int H>
__global__ __launch_bounds__(GroupGeom<G>::BSZ) void k_crows_lds(
    LevelView L, const i32 *__restrict__ nodes, i64 count, const i32 *__restrict__ lab,
    int bits, u64 *__restrict__ rec_key, i32 *__restrict__ rec_w, i32 *__restrict__ cnt)
{
    constexpr int NGc = GroupGeom<G>::NG;
    __shared__ i32 s_key[NGc * H];
    __shared__ i32 s_val[NGc * H];
    __shared__ i64 red[32];
    GROUP_PROLOGUE(G)
    i32 *keys = s_key + gi * H;
    i32 *vals = s_val + gi * H;
    for (int s = gl; s < H; s += G) {
        keys[s] = -1;
        vals[s] = 0;
    }
    // rows labelled -1 belong to graphs leaving a batch: no records
    const bool keep = valid && lab[node] >= 0;
    group_sync<G>();
    if (keep) {
        const i64 e1 = L.rp[node + 1];
        for (i64 j = L.rp[node] + gl; j < e1; j += G) {
            int2 ed = L.e[j];
            const i32 c = lab[ed.x];
            u32 h = slot_of<H>(c);
            for (int probe = 0; probe < H; probe++) {
                i32 old = atomicCAS(&keys[h], -1, c);
                if (old == -1 || old == c) {
                    atomicAdd(&vals[h], ed.y);
                    break;
                }
                h = (h + 1) & (H - 1);
            }
        }
    }
    group_sync<G>();
    int mine = 0;
    if (keep)
        for (int s = gl; s < H; s += G) mine += keys[s] >= 0;
    int total;
    int pos = gscan<G>(mine, total, red);
    if (keep) {
        const u64 hi = (u64)(u32)lab[node] << bits;
        const i64 base = L.rp[node];
        for (int s = gl; s < H; s += G) {
            const i32 c = keys[s];
            if (c >= 0) {
                rec_key[base + pos] = hi | (u64)(u32)c;
                rec_w[base + pos] = vals[s];
                pos++;
            }
        }
        if (gl == 0) cnt[node] = total;
    }
}

// ------------------------------------------------------------------ hub rows
// One workgroup per chunk of a hub row.
__global__ __launch_bounds__(SLM_BS) void k_hub_zero(const i32 *__restrict__ hub_node, i32 nhub,
                                                    i32 *__restrict__ a, i32 *__restrict__ b)
{
    i32 h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < nhub) {
        a[hub_node[h]] = 0;
        if (b) b[hub_node[h]] = 0;
    }
}

__global__ __launch_bounds__(SLM_BS) void k_hub_strength(
    const i64 *__restrict__ rp, const int2 *__restrict__ e, const i32 *__restrict__ hub_node,
    const i32 *__restrict__ chunk_hub, const i64 *__restrict__ chunk_beg, i32 *__restrict__ k,
    i32 *__restrict__ diag)
{
    __shared__ i64 red[32];
    const i32 h = chunk_hub[blockIdx.x];
    const i32 node = hub_node[h];
    const i64 b = chunk_beg[blockIdx.x];
    i64 end = b + HUB_CHUNK;
    if (end > rp[node + 1]) end = rp[node + 1];
    i64 s = 0, d = 0;
    for (i64 j = b + threadIdx.x; j < end; j += blockDim.x) {
        int2 ed = e[j];
        s += ed.y;
        if (ed.x == node) d += ed.y;
    }
    s = block_sum<i64>(s, red);
    d = block_sum<i64>(d, red);
    if (threadIdx.x == 0) {
        atomicAdd(&k[node], (i32)s);
        if (d) atomicAdd(&diag[node], (i32)d);
    }
}

template <bool REPOINT>
__global__ __launch_bounds__(SLM_BS) void k_hub_argmax(
    LevelView L, const i32 *__restrict__ hub_node, const i32 *__restrict__ chunk_hub,
    const i64 *__restrict__ chunk_beg, const i32 *__restrict__ lab,
    const i32 *__restrict__ best_c, const uint8_t *__restrict__ accept,
    i64 *__restrict__ chunk_key, i32 *__restrict__ chunk_id)
{
    __shared__ i64 red[32];
    const i32 h = chunk_hub[blockIdx.x];
    const i32 node = hub_node[h];
    bool active = true;
    if constexpr (REPOINT) active = accept[node] != 0;
    i64 bk = INT64_MIN;
    i32 bj = INT32_MAX;
    if (active) {
        const i64 b = chunk_beg[blockIdx.x];
        i64 end = b + HUB_CHUNK;
        if (end > L.rp[node + 1]) end = L.rp[node + 1];
        const i64 ki = L.k[node];
        const i64 yi = node_y(L, node);
        const i64 m2 = node_m2(L, node);
        const i32 D = REPOINT ? best_c[node] : 0;
        for (i64 j = b + threadIdx.x; j < end; j += blockDim.x) {
            int2 ed = L.e[j];
            const i32 v = ed.x;
            if (v == node) continue;
            if (REPOINT && lab[v] != D) continue;
            i64 key = m2 * (i64)ed.y - ki * (i64)L.k[v] + yi * node_y(L, v);
            if (better_key(key, v, bk, bj)) {
                bk = key;
                bj = v;
            }
        }
    }
    block_best(bk, bj, red);
    if (threadIdx.x == 0) {
        chunk_key[blockIdx.x] = bk;
        chunk_id[blockIdx.x] = bj;
    }
}

template <bool REPOINT>
__global__ __launch_bounds__(SLM_BS) void k_hub_argmax_final(
    const i32 *__restrict__ hub_node, const i32 *__restrict__ chunk_first,
    const uint8_t *__restrict__ accept, const i64 *__restrict__ chunk_key,
    const i32 *__restrict__ chunk_id, i32 *__restrict__ a, int *__restrict__ err)
{
    __shared__ i64 red[32];
    const i32 h = blockIdx.x;
    const i32 node = hub_node[h];
    if (REPOINT && !accept[node]) return;  // uniform over the workgroup
    i64 bk = INT64_MIN;
    i32 bj = INT32_MAX;
    for (i32 c = chunk_first[h] + threadIdx.x; c < chunk_first[h + 1]; c += blockDim.x)
        if (better_key(chunk_key[c], chunk_id[c], bk, bj)) {
            bk = chunk_key[c];
            bj = chunk_id[c];
        }
    block_best(bk, bj, red);
    if (threadIdx.x == 0) write_assign<REPOINT>(a, node, bk, bj, err);
}

__global__ __launch_bounds__(SLM_BS) void k_hub_own(
    LevelView L, const i32 *__restrict__ hub_node, const i32 *__restrict__ chunk_hub,
    const i64 *__restrict__ chunk_beg, const i32 *__restrict__ lab,
    const uint8_t *__restrict__ active, i32 *__restrict__ wc)
{
    __shared__ i64 red[32];
    const i32 h = chunk_hub[blockIdx.x];
    const i32 node = hub_node[h];
    const i32 ci = lab[node];
    if (active && !active[ci]) return;  // uniform
    const i64 b = chunk_beg[blockIdx.x];
    i64 end = b + HUB_CHUNK;
    if (end > L.rp[node + 1]) end = L.rp[node + 1];
    i64 s = 0;
    for (i64 j = b + threadIdx.x; j < end; j += blockDim.x) {
        int2 ed = L.e[j];
        if (lab[ed.x] == ci) s += ed.y;
    }
    s = block_sum<i64>(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(&wc[node], (i32)s);
}

__global__ __launch_bounds__(SLM_BS) void k_hub_own_zero(const i32 *__restrict__ hub_node,
                                                        i32 nhub, const i32 *__restrict__ lab,
                                                        const uint8_t *__restrict__ active,
                                                        i32 *__restrict__ wc)
{
    i32 h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < nhub) {
        i32 node = hub_node[h];
        if (!active || active[lab[node]]) wc[node] = 0;
    }
}

// Hub contraction rows: one record per entry (merged later by the sort).
__global__ __launch_bounds__(SLM_BS) void k_hub_crows(
    LevelView L, const i32 *__restrict__ hub_node, const i32 *__restrict__ chunk_hub,
    const i64 *__restrict__ chunk_beg, const i32 *__restrict__ lab, int bits,
    u64 *__restrict__ rec_key, i32 *__restrict__ rec_w, i32 *__restrict__ cnt)
{
    const i32 h = chunk_hub[blockIdx.x];
    const i32 node = hub_node[h];
    const i64 b = chunk_beg[blockIdx.x];
    i64 end = b + HUB_CHUNK;
    if (end > L.rp[node + 1]) end = L.rp[node + 1];
    if (lab[node] < 0) return;  // the hub's graph leaves a batch: no records
    const u64 hi = (u64)(u32)lab[node] << bits;
    for (i64 j = b + threadIdx.x; j < end; j += blockDim.x) {
        int2 ed = L.e[j];
        rec_key[j] = hi | (u64)(u32)lab[ed.x];
        rec_w[j] = ed.y;
    }
    if (b == L.rp[node] && threadIdx.x == 0) cnt[node] = (i32)(L.rp[node + 1] - L.rp[node]);
}

// ------------------------------------------------------------------ bins
__device__ __forceinline__ int bin_of_degree(i64 d)
{
    if (d == 0) return BIN_ZERO;
    if (d <= 8) return BIN_8;
    if (d <= 32) return BIN_32;
    if (d <= 64) return BIN_64;
    if (d <= 128) return BIN_128;
    if (d <= 256) return BIN_256;
    if (d <= 512) return BIN_512;
    if (d <= 1024) return BIN_1024;
    if (d <= 2048) return BIN_2048;
    if (d <= 4096) return BIN_4096;
    return BIN_HUB;
}

// Bins are filled without global atomics and in increasing node order: per
// workgroup of SLM_BS nodes, the count of each bin (bin-major:
// cnt[b * nblk + workgroup]); an exclusive scan of these counts gives every
// workgroup's first slot in every bin.
__global__ __launch_bounds__(SLM_BS) void k_bin_count(const i64 *__restrict__ rp, i64 n,
                                                     i64 nblk, i64 *__restrict__ cnt)
{
    __shared__ int c[NBINS];
    if (threadIdx.x < NBINS) c[threadIdx.x] = 0;
    __syncthreads();
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&c[bin_of_degree(rp[i + 1] - rp[i])], 1);
    __syncthreads();
    if (threadIdx.x < NBINS) cnt[threadIdx.x * nblk + blockIdx.x] = c[threadIdx.x];
}

// off[b] = first slot of bin b (from the scanned counts), off[NBINS] = n.
__global__ void k_bin_bounds(const i64 *__restrict__ scanned, i64 nblk, i64 *__restrict__ off)
{
    const int b = threadIdx.x;
    if (b <= NBINS) off[b] = scanned[(i64)b * nblk];
}

// Row descriptors in bin order: one coalesced load gives a row its node, its
// degree and its first entry.
__global__ void k_rowdesc(const i32 *__restrict__ nodes, const i64 *__restrict__ rp, i64 n,
                          int4 *__restrict__ rowd)
{
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (i64)gridDim.x * blockDim.x) {
        const i32 u = nodes[t];
        const i64 b = rp[u];
        rowd[t] = make_int4(u, (i32)(rp[u + 1] - b), (i32)(u32)(b & 0xffffffffll),
                            (i32)(b >> 32));
    }
}

void launch_rowdesc(const i32 *nodes, const i64 *rp, i64 n, int4 *rowd, hipStream_t s)
{
    if (n <= 0) return;
    i64 g = (n + SLM_BS - 1) / SLM_BS;
    if (g > 16384) g = 16384;
    k_rowdesc<<<(unsigned)g, SLM_BS, 0, s>>>(nodes, rp, n, rowd);
}

// Node i goes to slot scanned[b * nblk + workgroup] + (its rank among the
// workgroup's nodes of bin b).
__global__ __launch_bounds__(SLM_BS) void k_bin_scatter(const i64 *__restrict__ rp, i64 n,
                                                       i64 nblk, const i64 *__restrict__ scanned,
                                                       i32 *__restrict__ bin_nodes)
{
    constexpr int NW = SLM_BS / 64;
    __shared__ int wc[NBINS][NW];
    const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    const int b = i < n ? bin_of_degree(rp[i + 1] - rp[i]) : -1;
    const int lane = threadIdx.x & 63, wid = threadIdx.x / 64;
    int rank = 0;
    for (int bb = 0; bb < NBINS; bb++) {
        const u64 mask = __ballot(b == bb);
        if (lane == 0) wc[bb][wid] = __popcll(mask);
        if (b == bb) rank = __popcll(mask & ((1ull << lane) - 1ull));
    }
    __syncthreads();
    if (b >= 0) {
        for (int w = 0; w < wid; w++) rank += wc[b][w];
        bin_nodes[scanned[(i64)b * nblk + blockIdx.x] + rank] = (i32)i;
    }
}

// span[2h], span[2h+1] = first and one-past-last entry of hub h's row.
__global__ void k_hub_degrees(const i64 *__restrict__ rp, const i32 *__restrict__ hub_node,
                              i32 nhub, i64 *__restrict__ span)
{
    i32 h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < nhub) {
        span[2 * h] = rp[hub_node[h]];
        span[2 * h + 1] = rp[hub_node[h] + 1];
    }
}

i64 bin_scan_elems(i64 n)
{
    const i64 m = NBINS * ((n + SLM_BS - 1) / SLM_BS);
    return 2 * (m + 1) + scan_tmp_elems(m + 1);
}

void launch_bins(const i64 *rp, i64 n, i64 *tmp, i64 *off_dev, i32 *bin_nodes, hipStream_t s)
{
    if (n <= 0) return;
    const i64 nblk = (n + SLM_BS - 1) / SLM_BS, m = NBINS * nblk;
    i64 *cnt = tmp, *scanned = tmp + (m + 1), *stmp = tmp + 2 * (m + 1);
    k_bin_count<<<(unsigned)nblk, SLM_BS, 0, s>>>(rp, n, nblk, cnt);
    launch_scan_i64(cnt, scanned, m, stmp, s);
    k_bin_bounds<<<1, 64, 0, s>>>(scanned, nblk, off_dev);
    k_bin_scatter<<<(unsigned)nblk, SLM_BS, 0, s>>>(rp, n, nblk, scanned, bin_nodes);
}
void launch_hub_degrees(const i64 *rp, const i32 *hub_node, i32 nhub, i64 *deg_out, hipStream_t s)
{
    if (nhub > 0) k_hub_degrees<<<grid_for(nhub, SLM_BS), SLM_BS, 0, s>>>(rp, hub_node, nhub, deg_out);
}

// ------------------------------------------------------------------ dispatch
template <int B>
static void bin_launch_geom(const Bins &Bn, i64 &count, const i32 *&nodes, unsigned &grid,
                            unsigned &block)
{
    constexpr int G = BinShape<B>::G;
    count = Bn.off[B + 1] - Bn.off[B];
    nodes = Bn.nodes + Bn.off[B];
    grid = grid_for(count, GroupGeom<G>::NG);
    block = GroupGeom<G>::BSZ;
}

#define FOR_LDS_BINS(X)                                                               \
    X(BIN_ZERO) X(BIN_8) X(BIN_32) X(BIN_64) X(BIN_128) X(BIN_256) X(BIN_512) X(BIN_1024)     \
    X(BIN_2048) X(BIN_4096)
// ASSIGN, re-pointing and own weights: rows of degree <= 64 in registers
// (bin, lanes per row, entries per lane), the others by lane-group loops
#define FOR_SHORT_BINS(X) X(BIN_8, 4, 2) X(BIN_32, 8, 4) X(BIN_64, 16, 4)
#define FOR_LONG_BINS(X)                                                              \
    X(BIN_ZERO) X(BIN_128) X(BIN_256) X(BIN_512) X(BIN_1024) X(BIN_2048) X(BIN_4096)

void run_strength_binned(const i64 *rp, const int2 *e, const Bins &Bn, i32 *k, i32 *diag,
                         hipStream_t s)
{
#define X(B)                                                                          \
    {                                                                                 \
        i64 cnt;                                                                      \
        const i32 *nd;                                                                \
        unsigned gr, bl;                                                              \
        bin_launch_geom<B>(Bn, cnt, nd, gr, bl);                                      \
        if (cnt > 0)                                                                  \
            k_strength<BinShape<B>::G><<<gr, bl, 0, s>>>(rp, e, nd, cnt, k, diag);         \
    }
    FOR_LDS_BINS(X)
#undef X
    if (Bn.nhub > 0) {
        k_hub_zero<<<grid_for(Bn.nhub, SLM_BS), SLM_BS, 0, s>>>(Bn.hub_node, Bn.nhub, k, diag);
        k_hub_strength<<<(unsigned)Bn.nchunk, SLM_BS, 0, s>>>(rp, e, Bn.hub_node, Bn.chunk_hub,
                                                             Bn.chunk_beg, k, diag);
    }
}

void run_assign(const LevelView &L, const Bins &Bn, i32 *a, i64 *hub_key, i32 *hub_id,
                hipStream_t s)
{
#define X(B)                                                                          \
    {                                                                                 \
        i64 cnt;                                                                      \
        const i32 *nd;                                                                \
        unsigned gr, bl;                                                              \
        bin_launch_geom<B>(Bn, cnt, nd, gr, bl);                                      \
        if (cnt > 0)                                                                  \
            k_argmax<BinShape<B>::G, false><<<gr, bl, 0, s>>>(L, nd, cnt, nullptr, nullptr, \
                                                              nullptr, a, nullptr);   \
    }
    FOR_LONG_BINS(X)
#undef X
#define X(B, G, U)                                                                    \
    {                                                                                 \
        const i64 cnt = Bn.off[B + 1] - Bn.off[B];                                    \
        if (cnt > 0)                                                                  \
            k_argmax_reg<G, U, false><<<grid_for(cnt, SLM_BS / G), SLM_BS, 0, s>>>(   \
                L, Bn.rowd + Bn.off[B], cnt, nullptr, nullptr, nullptr, a, nullptr);  \
    }
    FOR_SHORT_BINS(X)
#undef X
    if (Bn.nhub > 0) {
        k_hub_argmax<false><<<(unsigned)Bn.nchunk, SLM_BS, 0, s>>>(
            L, Bn.hub_node, Bn.chunk_hub, Bn.chunk_beg, nullptr, nullptr, nullptr, hub_key, hub_id);
        k_hub_argmax_final<false><<<(unsigned)Bn.nhub, SLM_BS, 0, s>>>(
            Bn.hub_node, Bn.chunk_off_of_hub, nullptr, hub_key, hub_id, a, nullptr);
    }
}

void run_repoint(const LevelView &L, const Bins &Bn, const i32 *lab, const i32 *best_c,
                 const uint8_t *accept, i32 *a, i64 *hub_key, i32 *hub_id, int *err,
                 hipStream_t s)
{
#define X(B)                                                                          \
    {                                                                                 \
        i64 cnt;                                                                      \
        const i32 *nd;                                                                \
        unsigned gr, bl;                                                              \
        bin_launch_geom<B>(Bn, cnt, nd, gr, bl);                                      \
        if (cnt > 0 && B != BIN_ZERO)                                                 \
            k_argmax<BinShape<B>::G, true><<<gr, bl, 0, s>>>(L, nd, cnt, lab, best_c, accept, a, \
                                                             err);                    \
    }
    FOR_LONG_BINS(X)
#undef X
#define X(B, G, U)                                                                    \
    {                                                                                 \
        const i64 cnt = Bn.off[B + 1] - Bn.off[B];                                    \
        if (cnt > 0)                                                                  \
            k_argmax_reg<G, U, true><<<grid_for(cnt, SLM_BS / G), SLM_BS, 0, s>>>(    \
                L, Bn.rowd + Bn.off[B], cnt, lab, best_c, accept, a, err);            \
    }
    FOR_SHORT_BINS(X)
#undef X
    if (Bn.nhub > 0) {
        k_hub_argmax<true><<<(unsigned)Bn.nchunk, SLM_BS, 0, s>>>(
            L, Bn.hub_node, Bn.chunk_hub, Bn.chunk_beg, lab, best_c, accept, hub_key, hub_id);
        k_hub_argmax_final<true><<<(unsigned)Bn.nhub, SLM_BS, 0, s>>>(
            Bn.hub_node, Bn.chunk_off_of_hub, accept, hub_key, hub_id, a, err);
    }
}

void run_own_weight(const LevelView &L, const Bins &Bn, const i32 *lab, const uint8_t *active,
                    i32 *wc, hipStream_t s)
{
#define X(B)                                                                          \
    {                                                                                 \
        i64 cnt;                                                                      \
        const i32 *nd;                                                                \
        unsigned gr, bl;                                                              \
        bin_launch_geom<B>(Bn, cnt, nd, gr, bl);                                      \
        if (cnt > 0) k_own<BinShape<B>::G><<<gr, bl, 0, s>>>(L, nd, cnt, lab, active, wc); \
    }
    FOR_LONG_BINS(X)
#undef X
#define X(B, G, U)                                                                    \
    {                                                                                 \
        const i64 cnt = Bn.off[B + 1] - Bn.off[B];                                    \
        if (cnt > 0)                                                                  \
            k_own_reg<G, U><<<grid_for(cnt, SLM_BS / G), SLM_BS, 0, s>>>(             \
                L, Bn.rowd + Bn.off[B], cnt, lab, active, wc);                        \
    }
    FOR_SHORT_BINS(X)
#undef X
    if (Bn.nhub > 0) {
        k_hub_own_zero<<<grid_for(Bn.nhub, SLM_BS), SLM_BS, 0, s>>>(Bn.hub_node, Bn.nhub, lab,
                                                                   active, wc);
        k_hub_own<<<(unsigned)Bn.nchunk, SLM_BS, 0, s>>>(L, Bn.hub_node, Bn.chunk_hub,
                                                        Bn.chunk_beg, lab, active, wc);
    }
}

void run_contract_rows(const LevelView &L, const Bins &Bn, const i32 *lab, int lab_bits,
                       u64 *rec_key, i32 *rec_w, i32 *cnt, hipStream_t s)
{
#define X(B)                                                                          \
    {                                                                                 \
        i64 c_;                                                                       \
        const i32 *nd;                                                                \
        unsigned gr, bl;                                                              \
        bin_launch_geom<B>(Bn, c_, nd, gr, bl);                                       \
        if (c_ > 0)                                                                   \
            k_crows_lds<BinShape<B>::G, BinShape<B>::H><<<gr, bl, 0, s>>>(            \
                L, nd, c_, lab, lab_bits, rec_key, rec_w, cnt);                       \
    }
    FOR_LDS_BINS(X)
#undef X
    if (Bn.nhub > 0)
        k_hub_crows<<<(unsigned)Bn.nchunk, SLM_BS, 0, s>>>(L, Bn.hub_node, Bn.chunk_hub,
                                                          Bn.chunk_beg, lab, lab_bits, rec_key,
                                                          rec_w, cnt);
}

// ------------------------------------------------------------------ row ids of the entries
template <int G>
__global__ __launch_bounds__(GroupGeom<G>::BSZ) void k_src(const i64 *__restrict__ rp,
                                                          const i32 *__restrict__ nodes,
                                                          i64 count, i32 *__restrict__ src)
{
    GROUP_PROLOGUE(G)
    if (valid)
        for (i64 j = rp[node] + gl; j < rp[node + 1]; j += G) src[j] = node;
}

__global__ __launch_bounds__(SLM_BS) void k_hub_src(const i64 *__restrict__ rp,
                                                   const i32 *__restrict__ hub_node,
                                                   const i32 *__restrict__ chunk_hub,
                                                   const i64 *__restrict__ chunk_beg,
                                                   i32 *__restrict__ src)
{
    const i32 node = hub_node[chunk_hub[blockIdx.x]];
    const i64 b = chunk_beg[blockIdx.x];
    i64 end = b + HUB_CHUNK;
    if (end > rp[node + 1]) end = rp[node + 1];
    for (i64 j = b + threadIdx.x; j < end; j += blockDim.x) src[j] = node;
}

void fill_src(const LevelView &L, const Bins &Bn, i32 *src, hipStream_t s)
{
#define X(B)                                                                          \
    {                                                                                 \
        i64 cnt;                                                                      \
        const i32 *nd;                                                                \
        unsigned gr, bl;                                                              \
        bin_launch_geom<B>(Bn, cnt, nd, gr, bl);                                      \
        if (cnt > 0 && B != BIN_ZERO) k_src<BinShape<B>::G><<<gr, bl, 0, s>>>(L.rp, nd, cnt, src); \
    }
    FOR_LDS_BINS(X)
#undef X
    if (Bn.nhub > 0)
        k_hub_src<<<(unsigned)Bn.nchunk, SLM_BS, 0, s>>>(L.rp, Bn.hub_node, Bn.chunk_hub,
                                                        Bn.chunk_beg, src);
}

i64 level_strengths(Work &W, const i64 *rp, const int2 *e, const Bins &B, i64 n, i32 *k,
                    i32 *diag, hipStream_t s)
{
    launch_fill_i64(W.counters, 0, 1, s);
    run_strength_binned(rp, e, B, k, diag, s);
    if (n > 0) {
        i64 g = (n + SLM_BS - 1) / SLM_BS;
        if (g > 1024) g = 1024;
        k_sum_i32<<<(unsigned)g, SLM_BS, 0, s>>>(k, n, W.counters);
    }
    read_scalars(W, W.counters, 1, s);
    return W.h_scal[0];
}
