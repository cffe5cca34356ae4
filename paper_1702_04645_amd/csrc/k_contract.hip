// AGGREGATE (Sec. 3.5): the community graph of the next level,
// A'_CD = sum of A_uv over u in C, v in D.  Rows are first pre-aggregated
// (one record per distinct (lab_u, lab_v) of a row), the records are sorted
// by the composite key lab_u << bits | lab_v with an LSD radix sort of 8-bit
// digits, equal keys are merged by a segmented sum, and the new row offsets
// come from a histogram of the row part of the keys.
#include "slm_forest.h"

#define RS_BINS 256
#define RS_SUB 16
#define RS_TILE (SLM_BS * RS_SUB)

#define FLAT_LOOP(n)                                                                  \
    for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j < (n);                 \
         j += (i64)gridDim.x * blockDim.x)

static unsigned flat_grid(i64 n)
{
    i64 g = (n + SLM_BS - 1) / SLM_BS;
    if (g > 16384) g = 16384;
    if (g < 1) g = 1;
    return (unsigned)g;
}

// Records of row u sit at [rp[u], rp[u] + cnt[u]); pack them at roff[u].
__global__ void k_compact_records(const i32 *__restrict__ src, const i64 *__restrict__ rp,
                                  const i32 *__restrict__ cnt, const i64 *__restrict__ roff,
                                  i64 nnz, const u64 *__restrict__ kin, const i32 *__restrict__ vin,
                                  u64 *__restrict__ kout, i32 *__restrict__ vout)
{
    FLAT_LOOP(nnz)
    {
        i32 u = src[j];
        i64 t = j - rp[u];
        if (t < cnt[u]) {
            kout[roff[u] + t] = kin[j];
            vout[roff[u] + t] = vin[j];
        }
    }
}

// ------------------------------------------------------------------ radix sort
// Tile of RS_TILE items: sub-round r covers items tile + r*256 + tid, so the
// tile is visited in order and the scatter below is stable.
__global__ __launch_bounds__(SLM_BS) void k_rs_hist(const u64 *__restrict__ keys, i64 n,
                                                   int shift, i64 nblk, i64 *__restrict__ hist)
{
    __shared__ int cnt[RS_BINS];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const i64 tile = (i64)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_SUB; r++) {
        i64 idx = tile + (i64)r * SLM_BS + threadIdx.x;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & (RS_BINS - 1)], 1);
    }
    __syncthreads();
    hist[(i64)threadIdx.x * nblk + blockIdx.x] = cnt[threadIdx.x];
}

__global__ __launch_bounds__(SLM_BS) void k_rs_scatter(const u64 *__restrict__ kin,
                                                      const i32 *__restrict__ vin, i64 n,
                                                      int shift, i64 nblk,
                                                      const i64 *__restrict__ offs,
                                                      u64 *__restrict__ kout,
                                                      i32 *__restrict__ vout)
{
    __shared__ i64 base[RS_BINS];
    __shared__ int run[RS_BINS];
    __shared__ int wcnt[SLM_BS / 64][RS_BINS];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid / 64;
    base[tid] = offs[(i64)tid * nblk + blockIdx.x];
    run[tid] = 0;
    const u64 lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const i64 tile = (i64)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_SUB; r++) {
        for (int w = 0; w < SLM_BS / 64; w++) wcnt[w][tid] = 0;
        __syncthreads();
        const i64 idx = tile + (i64)r * SLM_BS + tid;
        const bool ok = idx < n;
        u64 key = ok ? kin[idx] : 0;
        i32 val = ok ? vin[idx] : 0;
        const int d = (int)((key >> shift) & (RS_BINS - 1));
        u64 peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1;
            const u64 m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const int rank = __popcll(peers & lt);
        if (ok && rank == 0) wcnt[wid][d] = __popcll(peers);
        __syncthreads();
        if (ok) {
            int before = run[d];
            for (int w = 0; w < wid; w++) before += wcnt[w][d];
            const i64 dst = base[d] + before + rank;
            kout[dst] = key;
            vout[dst] = val;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < SLM_BS / 64; w++) add += wcnt[w][tid];
        run[tid] += add;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ merge and rows
__global__ void k_seg_heads(const u64 *__restrict__ keys, i64 n, uint8_t *__restrict__ head)
{
    FLAT_LOOP(n) head[j] = (j == 0 || keys[j] != keys[j - 1]) ? 1 : 0;
}

// The head of segment s (record j, s = hpos[j]) writes the segment's key and
// its first record; start[u] = n closes the last segment.
__global__ void k_seg_starts(const u64 *__restrict__ keys, i64 n, const uint8_t *__restrict__ head,
                             const i64 *__restrict__ hpos, i64 u, u64 *__restrict__ ukey,
                             i32 *__restrict__ start)
{
    FLAT_LOOP(n)
    {
        if (head[j]) {
            ukey[hpos[j]] = keys[j];
            start[hpos[j]] = (i32)j;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[u] = (i32)n;
}

// Weight of segment s from the exclusive prefix sums P of the sorted
// records' weights: P[start[s+1]] - P[start[s]] (no atomics: equal keys are
// adjacent after the sort).
__global__ void k_seg_sums(const i64 *__restrict__ P, const i32 *__restrict__ start, i64 u,
                           i32 *__restrict__ uw)
{
    FLAT_LOOP(u) uw[j] = (i32)(P[start[j + 1]] - P[start[j]]);
}

// Row offsets of the sorted unique keys: rp[r] = the first key whose row is
// at least r.  Key j writes the rows after the previous key's row up to its
// own (rows without an entry included); j = u closes the rows up to nrows.
__global__ void k_row_ptr(const u64 *__restrict__ ukey, i64 u, int bits, i64 nrows,
                          i64 *__restrict__ rp)
{
    for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j <= u;
         j += (i64)gridDim.x * blockDim.x) {
        const i64 r0 = j == 0 ? 0 : (i64)(ukey[j - 1] >> bits) + 1;
        const i64 r1 = j == u ? nrows : (i64)(ukey[j] >> bits);
        for (i64 r = r0; r <= r1; r++) rp[r] = j;
    }
}

__global__ void k_emit_entries(const u64 *__restrict__ ukey, const i32 *__restrict__ uw, i64 u,
                               int bits, int2 *__restrict__ e_out)
{
    const u64 mask = (bits >= 64) ? ~0ull : ((1ull << bits) - 1ull);
    FLAT_LOOP(u) e_out[j] = make_int2((i32)(ukey[j] & mask), uw[j]);
}

static int bits_for(i64 nc)
{
    int b = 1;
    while (((i64)1 << b) < nc) b++;
    return b;
}

// Sorts (keys, vals) of n items on their low `bits` bits; returns the buffers
// that hold the result (either the inputs or the alternates).
static void radix_sort(Work &W, u64 *&k, i32 *&v, u64 *&k2, i32 *&v2, i64 n, int bits,
                       hipStream_t s)
{
    const i64 nblk = (n + RS_TILE - 1) / RS_TILE;
    const i64 hn = nblk * RS_BINS;
    if (hn + 1 > W.hist_cap) {
        if (W.hist) {
            HIPCHK(hipStreamSynchronize(s));
            W.dm->put(W.hist, sizeof(i64) * 2 * (size_t)W.hist_cap);
        }
        W.hist = nullptr;
        W.hist_cap = 0;
        const i64 cap = hn + 1 + 4096;
        W.hist = (i64 *)W.dm->get(sizeof(i64) * 2 * (size_t)cap);
        W.hist_cap = cap;
    }
    i64 *hist = W.hist, *offs = W.hist + W.hist_cap;
    i64 *tmp = W.scan_tmp;  // scan_tmp is sized for n0 + nnz0
    for (int shift = 0; shift < bits; shift += 8) {
        k_rs_hist<<<(unsigned)nblk, SLM_BS, 0, s>>>(k, n, shift, nblk, hist);
        launch_scan_i64(hist, offs, hn, tmp, s);
        k_rs_scatter<<<(unsigned)nblk, SLM_BS, 0, s>>>(k, v, n, shift, nblk, offs, k2, v2);
        u64 *tk = k;
        k = k2;
        k2 = tk;
        i32 *tv = v;
        v = v2;
        v2 = tv;
    }
}

// Records (row << bits | column, weight) in (k, v), alternates (k2, v2): the
// CSR of nrows rows that sums the weights of equal keys, rows sorted by
// column.  Returns its entry count.
static i64 records_to_csr(Work &W, u64 *k, i32 *v, u64 *k2, i32 *v2, i64 recs, int bits,
                          i64 nrows, i64 *rp_out, int2 *e_out, hipStream_t s)
{
    if (recs > 0) radix_sort(W, k, v, k2, v2, recs, 2 * bits, s);
    // merge equal keys: heads -> segment starts and keys (into k2, v2) ->
    // prefix sums of the weights (into rank_e, once the head positions are
    // used) -> segment sums (into v)
    uint8_t *head = W.head_e;
    i64 *hpos = W.rank_e;
    i64 uniq = 0;
    if (recs > 0) {
        k_seg_heads<<<flat_grid(recs), SLM_BS, 0, s>>>(k, recs, head);
        launch_scan_u8(head, hpos, recs, W.scan_tmp, s);
        read_scalars(W, hpos + recs, 1, s);
        uniq = W.h_scal[0];
        k_seg_starts<<<flat_grid(recs), SLM_BS, 0, s>>>(k, recs, head, hpos, uniq, k2, v2);
        i64 *P = W.rank_e;
        launch_scan_i32(v, P, recs, W.scan_tmp, s);
        k_seg_sums<<<flat_grid(uniq), SLM_BS, 0, s>>>(P, v2, uniq, v);
    }
    // rows of the result (no atomics: the keys are sorted by row)
    k_row_ptr<<<flat_grid(uniq + 1), SLM_BS, 0, s>>>(k2, uniq, bits, nrows, rp_out);
    if (uniq > 0) k_emit_entries<<<flat_grid(uniq), SLM_BS, 0, s>>>(k2, v, uniq, bits, e_out);
    return uniq;
}

i64 contract_level(Work &W, const LevelView &Lv, const Bins &B, const i32 *lab, i64 nc,
                   i64 *rp_out, int2 *e_out, hipStream_t s)
{
    const i64 n = Lv.n, nnz = Lv.nnz;
    const int bits = bits_for(nc);
    launch_fill_i32(W.cnt, 0, n, s);
    run_contract_rows(Lv, B, lab, bits, W.rk0, W.rv0, W.cnt, s);
    launch_scan_i32(W.cnt, W.roff, n, W.scan_tmp, s);
    read_scalars(W, W.roff + n, 1, s);
    const i64 recs = W.h_scal[0];
    if (nnz > 0)
        k_compact_records<<<flat_grid(nnz), SLM_BS, 0, s>>>(W.src, Lv.rp, W.cnt, W.roff, nnz,
                                                          W.rk0, W.rv0, W.rk1, W.rv1);
    return records_to_csr(W, W.rk1, W.rv1, W.rk0, W.rv0, recs, bits, nc, rp_out, e_out, s);
}

// Both records (u, v, w) and (v, u, w) of every entry of row u; one thread
// per row.
__global__ void k_sym_records(const i64 *__restrict__ rp, const int2 *__restrict__ e, i64 n,
                              int bits, u64 *__restrict__ kout, i32 *__restrict__ vout)
{
    for (i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (i64)gridDim.x * blockDim.x) {
        for (i64 j = rp[u]; j < rp[u + 1]; j++) {
            const int2 ed = e[j];
            kout[2 * j] = ((u64)u << bits) | (u64)(u32)ed.x;
            kout[2 * j + 1] = ((u64)(u32)ed.x << bits) | (u64)u;
            vout[2 * j] = ed.y;
            vout[2 * j + 1] = ed.y;
        }
    }
}

// y[u] = sum of the row of u minus the sum of its column (k_out - k_in) of
// the directed matrix in (rp, e).
__global__ void k_out_minus_in(const i64 *__restrict__ rp, const int2 *__restrict__ e, i64 n,
                               i32 *__restrict__ y)
{
    for (i64 u = (i64)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (i64)gridDim.x * blockDim.x) {
        i64 out = 0;
        for (i64 j = rp[u]; j < rp[u + 1]; j++) {
            const int2 ed = e[j];
            out += ed.y;
            atomicSub(&y[ed.x], ed.y);
        }
        atomicAdd(&y[u], (i32)out);
    }
}

i64 symmetrize_level(Work &W, i64 *rp, int2 *e, i64 n, i64 nnz, i32 *y, hipStream_t s)
{
    launch_fill_i32(y, 0, n, s);
    if (n > 0) k_out_minus_in<<<flat_grid(n), SLM_BS, 0, s>>>(rp, e, n, y);
    const int bits = bits_for(n);
    if (n > 0) k_sym_records<<<flat_grid(n), SLM_BS, 0, s>>>(rp, e, n, bits, W.rk0, W.rv0);
    return records_to_csr(W, W.rk0, W.rv0, W.rk1, W.rv1, 2 * nnz, bits, n, rp, e, s);
}
