// Internal declarations of the gfx950 implementation of the Synchronised
// Louvain Method.  Device helpers, the level view handed to kernels, and the
// host-side launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

typedef int64_t i64;
typedef int32_t i32;
typedef uint32_t u32;
typedef uint64_t u64;

#define SLM_WAVE 64
#define SLM_BS 256

// ---------------------------------------------------------------- errors
struct SlmError {
    int status;
    std::string msg;
};
#define HIPCHK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw SlmError{4, std::string(#call) + ": " + hipGetErrorString(e_)};     \
    } while (0)

// ---------------------------------------------------------------- device memory
// Every device buffer of a handle comes from here: the caller's allocator
// (alloc/free callbacks with an opaque context, told the handle's stream)
// when one was given at creation, else hipMalloc / hipFree.  get() throws
// SlmError{SLM_E_NOMEM} when the allocator returns null; put() never throws.
// Buffers that grow are released only after the handle's stream is idle, so
// a stream-ordered allocator may hand the memory to other work at once.
struct DevMem {
    void *ctx = nullptr;
    void *(*fn_alloc)(void *ctx, size_t bytes, void *stream) = nullptr;
    void (*fn_free)(void *ctx, void *p, void *stream) = nullptr;
    hipStream_t s = nullptr;
    i64 held = 0;  // bytes currently held
    void *get(size_t bytes);
    void put(void *p, size_t bytes);
};

// Grows a device buffer of `cap` elements to at least `need` (new capacity
// need * 1.5 + pad); the old contents are dropped.
template <typename T>
static void dm_grow(DevMem &dm, T *&p, i64 &cap, i64 need, i64 pad)
{
    if (need <= cap) return;
    if (p) {
        HIPCHK(hipStreamSynchronize(dm.s));
        dm.put(p, sizeof(T) * (size_t)cap);
    }
    p = nullptr;
    cap = 0;
    const i64 c = need + need / 2 + pad;
    p = (T *)dm.get(sizeof(T) * (size_t)c);
    cap = c;
}

// ---------------------------------------------------------------- degree bins
// A node is handled by a group of lanes sized to its degree.  Bins 1..6 keep
// the per-node community table in LDS; bin 7 ("hub") rows are split in
// chunks of HUB_CHUNK entries spread over many workgroups, with the table in
// HBM.  Bin 0 holds isolated nodes.
enum {
    BIN_ZERO = 0, BIN_8, BIN_32, BIN_64, BIN_128, BIN_256, BIN_512, BIN_1024, BIN_2048, BIN_4096,
    BIN_HUB, NBINS
};
static const i64 kBinMaxDeg[NBINS] = {0, 8, 32, 64, 128, 256, 512, 1024, 2048, 4096, INT64_MAX};
#define HUB_CHUNK 2048
#define HUB_PART 1024  // distinct labels expected in one partition of a hub row
#define HUB_PMAX 1024  // partitions of one hub row at most
#define HUB_TH 2048    // LDS slots of a partition table
#define HUB_TCAP 1536  // pairs a partition table takes in one pass

// Work item of the sweep's hub chunk kernel: entries [beg, end) of hub row
// `node`; its distinct labels go to pairs [out ..) and its partition offsets
// to [pbase, pbase + 2^logp].
struct HubChunk {
    i64 beg, end, out, pbase;
    i32 node, logp, pad0, pad1;
};
// Work item of the hub partition kernel: partition p of hub row `node`,
// whose nch chunks (from c0) keep their offsets from pbase0 on, 2^logp + 1
// per chunk.
struct HubTile {
    i64 pbase0;
    i32 node, c0, nch, logp, p, pad;
};

struct Bins {
    i32 *nodes = nullptr;      // device: node ids grouped by bin
    i64 off[NBINS + 1] = {0};  // host: bin b = nodes[off[b] .. off[b+1])
    // hub rows: chunks of HUB_CHUNK entries, and 2^logp label partitions
    // ("tiles") per hub
    i32 nhub = 0;
    i64 nchunk = 0;
    i64 hub_entries = 0;       // sum of the hubs' degrees
    i64 npoff = 0;             // sum over chunks of (partitions of its hub + 1)
    i32 *hub_node = nullptr;   // device [nhub]
    i32 *chunk_hub = nullptr;  // device [nchunk] hub index of each chunk
    i64 *chunk_beg = nullptr;  // device [nchunk] first entry of each chunk
    HubChunk *hchunk = nullptr;// device [nchunk]
    i32 *chunk_off_of_hub = nullptr; // device [nhub+1] first chunk of each hub
    i64 ntile = 0;             // partitions over all hubs
    HubTile *htile = nullptr;  // device [ntile]
    i32 *tile_off_of_hub = nullptr; // device [nhub+1] first partition of each hub
    int hub_cap = HUB_TCAP;    // pairs per pass of a partition table
    int hub_tbits = 11;        // log2 of the partition table's slots (<= log2 HUB_TH)
    // workgroups of the persistent sweep kernel of each bin (0: the default)
    i32 grid_cap[NBINS] = {0};
    i64 *span = nullptr;       // device [2*nhub] entry range of each hub
    int4 *rowd = nullptr;      // device [n] per node in bin order: (node, degree,
                               // first entry low 32 bits, high 32 bits)
    int2 *ls = nullptr;        // device [n] scratch of the sweep: (label, S_label)
    // capacities of the arrays above: they only grow, so setting up a level
    // frees nothing (a free would synchronise the whole device)
    i64 cap_chunk_hub = 0, cap_chunk_beg = 0, cap_hchunk = 0, cap_chunk_off = 0, cap_htile = 0,
        cap_tile_off = 0, cap_span = 0;
};

// Read-only view of one level's graph as the kernels see it.
struct LevelView {
    const i64 *rp;   // n+1 offsets
    const int2 *e;   // nnz entries: x = column, y = weight
    const i32 *k;    // strengths (the null model's x; the row sums by default)
    const i32 *diag; // A_ii (0 if absent)
    // Second strength of the directed model and its community totals (null
    // otherwise): every gain A*w - x_i*X_C gains + y_i*Y_C.  sy holds the
    // totals of the labelling the current step works on.
    const i32 *y;
    const i32 *sy;
    i64 n;
    i64 nnz;
    i64 m2;  // scale A of the edge term (M2 for the default model)
    // A batch is the disjoint union of independent graphs.  Every key of a
    // node then uses the total weight of its own graph, and the acceptance
    // draw uses its graph's seed, level and local node number.  All null for
    // a single graph (m2 above applies to every node).
    const i32 *m2n;   // per node: M2 of its graph
    const i32 *gid;   // per node: graph index
    const i64 *gbase; // per graph: first node at this level
    const u64 *gseed; // per graph: seed
    const i32 *glev;  // per graph: level index
};

__device__ __forceinline__ i64 node_m2(const LevelView &L, i64 i)
{
    return L.m2n ? (i64)L.m2n[i] : L.m2;
}

// y_i, and Y_C of community c, of the directed model (0 for the others).
__device__ __forceinline__ i64 node_y(const LevelView &L, i64 i)
{
    return L.y ? (i64)L.y[i] : 0;
}
__device__ __forceinline__ i64 comm_y(const LevelView &L, i32 c)
{
    return L.y ? (i64)L.sy[c] : 0;
}

// Adds v to acc[key] for every lane of the wavefront, where the keys are
// non-decreasing across lanes (nodes of one graph are contiguous): a
// segmented reduction leaves one atomic per distinct key.  Only trailing
// lanes (past the end of the range) may pass key < 0; a lane inside the range
// that adds nothing passes its own key with v = 0.  Every lane of the
// wavefront must call it.
__device__ __forceinline__ void seg_add_sorted(unsigned long long *acc, i32 key, i64 v)
{
    const int lane = threadIdx.x & 63;
    i64 x = key >= 0 ? v : 0;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const i64 y = __shfl_up(x, d, 64);
        const i32 ky = __shfl_up(key, d, 64);
        if (lane >= d && ky == key) x += y;
    }
    const i32 kn = __shfl_down(key, 1, 64);
    const bool last = lane == 63 || kn != key;
    if (last && key >= 0 && x != 0) atomicAdd(&acc[key], (unsigned long long)x);
}

// ---------------------------------------------------------------- device helpers
__device__ __forceinline__ bool better_key(i64 k1, i32 id1, i64 k2, i32 id2)
{
    return k1 > k2 || (k1 == k2 && id1 < id2);
}

__device__ __forceinline__ u32 hash_label(i32 c)
{
    return (u32)c * 0x9E3779B1u;
}

// Sum over a group of G lanes (G a power of two, at most 64).
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// Best (key desc, id asc) over a group of G lanes (G <= 64).
template <int G>
__device__ __forceinline__ void group_best(i64 &key, i32 &id)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        i64 ok = __shfl_xor(key, off, G);
        i32 oi = __shfl_xor(id, off, G);
        if (better_key(ok, oi, key, id)) {
            key = ok;
            id = oi;
        }
    }
}

// Workgroup-wide best (key desc, id asc); every thread gets the result.
// scratch: at least 2 * (blockDim/64) slots of i64.
__device__ __forceinline__ void block_best(i64 &key, i32 &id, i64 *scratch)
{
    group_best<64>(key, id);
    const int wid = threadIdx.x / 64, nw = blockDim.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        scratch[2 * wid] = key;
        scratch[2 * wid + 1] = id;
    }
    __syncthreads();
    key = scratch[0];
    id = (i32)scratch[1];
    for (int w = 1; w < nw; w++) {
        i64 k2 = scratch[2 * w];
        i32 i2 = (i32)scratch[2 * w + 1];
        if (better_key(k2, i2, key, id)) {
            key = k2;
            id = i2;
        }
    }
    __syncthreads();
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, i64 *scratch)
{
    v = group_sum<64>(v);
    const int wid = threadIdx.x / 64, nw = blockDim.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[wid] = (i64)v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < nw; w++) s += (T)scratch[w];
    __syncthreads();
    return s;
}

static inline unsigned grid_for(i64 items, int per_block)
{
    i64 g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// ---------------------------------------------------------------- utilities (k_util.hip)
void launch_fill_i32(i32 *p, i32 v, i64 n, hipStream_t s);
void launch_scale_i32(i32 *p, i32 f, i64 n, hipStream_t s);  // p[i] *= f
void launch_fill_i64(i64 *p, i64 v, i64 n, hipStream_t s);
void launch_fill_u8(uint8_t *p, uint8_t v, i64 n, hipStream_t s);
void launch_iota_i32(i32 *p, i64 n, hipStream_t s);
// out[0..n] = exclusive prefix sums of in[0..n-1], out[n] = total.
// tmp: at least scan_tmp_elems(n) i64.
i64 scan_tmp_elems(i64 n);
void launch_scan_i32(const i32 *in, i64 *out, i64 n, i64 *tmp, hipStream_t s);
void launch_scan_i64(const i64 *in, i64 *out, i64 n, i64 *tmp, hipStream_t s);
void launch_scan_u8(const uint8_t *in, i64 *out, i64 n, i64 *tmp, hipStream_t s);

// ---------------------------------------------------------------- level setup (k_rows.hip)
// Degree bins: bin_nodes = the nodes of bin 0, then bin 1, ..., each in
// increasing order; off_dev[0..NBINS] = the bins' first slots and n.  tmp
// holds bin_scan_elems(n) i64.
i64 bin_scan_elems(i64 n);
void launch_bins(const i64 *rp, i64 n, i64 *tmp, i64 *off_dev, i32 *bin_nodes, hipStream_t s);
void launch_rowdesc(const i32 *nodes, const i64 *rp, i64 n, int4 *rowd, hipStream_t s);
// span_out[2h], span_out[2h+1] = entry range of hub h's row.
void launch_hub_degrees(const i64 *rp, const i32 *hub_node, i32 nhub, i64 *span_out,
                        hipStream_t s);

// ---------------------------------------------------------------- row kernels (k_rows.hip)
// ASSIGN (Sec. 3.1): a[i] = best neighbour or i.
void run_assign(const LevelView &L, const Bins &B, i32 *a, i64 *hub_key, i32 *hub_id,
                hipStream_t s);
// Side streams of a handle: the degree bins of a sweep are independent, so
// they run concurrently (fork after the work already queued on the main
// stream, join before anything after them).
#define FAN_SIDE 3
#define FAN_MIN_ENTRIES ((i64)1 << 22)  // smaller levels: the fork costs more than it saves
struct Fanout {
    hipStream_t side[FAN_SIDE] = {nullptr, nullptr, nullptr};
    hipEvent_t fork = nullptr, join[FAN_SIDE] = {nullptr, nullptr, nullptr};
    i64 min_entries = FAN_MIN_ENTRIES;  // levels with fewer entries stay on one stream
    // the fan-out to use for a level of nnz entries (null: one stream)
    const Fanout *use(i64 nnz) const { return side[0] && nnz >= min_entries ? this : nullptr; }
};
// MAXIMAL sweep (Sec. 3.4): best_c, delta, w_own from labels and totals.
// Hub scratch: hub_part [hub_entries] pairs, hub_poff [npoff], hub_cwin
// [nchunk], hub_tile_key / hub_tile_id [ntile].  F may be null (all bins on s).
void run_sweep(const LevelView &L, const Bins &B, const i32 *lab, const i32 *sigma,
               i32 *best_c, i64 *delta, i32 *w_own, int2 *hub_part, i64 *hub_poff,
               i32 *hub_cwin, i64 *hub_tile_key, i32 *hub_tile_id, hipStream_t s,
               const Fanout *F);
// wc[i] = sum of A_ij over j with lab[j] == lab[i] (diagonal included); only
// for nodes with active[lab[i]] != 0 when active is given.
void run_own_weight(const LevelView &L, const Bins &B, const i32 *lab, const uint8_t *active,
                    i32 *wc, hipStream_t s);
// Re-pointing (Sec. 3.4): for nodes with accept[i], a[i] = argmax over
// neighbours j with lab[j] == best_c[i] of pair(i,j), ties to the lowest j.
// err (device int, may be null) is set when an accepted node has no
// neighbour in its target community; that node's pointer is then unchanged.
void run_repoint(const LevelView &L, const Bins &B, const i32 *lab, const i32 *best_c,
                 const uint8_t *accept, i32 *a, i64 *hub_key, i32 *hub_id, int *err,
                 hipStream_t s);
// Contraction records of every row: distinct (lab_u, lab_v) pairs with summed
// weights, written at rec_key/rec_w[rp[u] ..]; cnt[u] = their number.
void run_contract_rows(const LevelView &L, const Bins &B, const i32 *lab, int lab_bits,
                       u64 *rec_key, i32 *rec_w, i32 *cnt, hipStream_t s);

