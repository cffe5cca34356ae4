// C ABI of include/slm.h: handles, validation, level state, and the level
// loop of Algorithm 1 (ASSIGN, COMPONENTS, POSITIVE, MAXIMAL rounds,
// AGGREGATE) driving the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <cstring>
#include <string>
#include <vector>

#include "slm.h"
#include "slm_forest.h"

#define REQUIRE(cond, code, msg)                                                      \
    do {                                                                              \
        if (!(cond)) throw SlmError{code, msg};                                       \
    } while (0)

static thread_local std::string g_err;

// The calling thread's last error message (also set by noalloc.hip).
std::string &slm_error_slot()
{
    return g_err;
}

struct slm_result {
    i64 n0 = 0;
    i64 t_submit_ns = 0, t_done_ns = 0;  // served requests: steady-clock times
    std::vector<i64> nc, nq;
    std::vector<double> q;
    std::vector<i32> rounds, conv;
    std::vector<std::vector<i32>> labels;
};

// One graph of a union.
struct Member {
    u64 ticket = 0;           // batch index, or server ticket
    i64 n0 = 0, nnz0 = 0, m2 = 0;
    u64 seed = 0;
    bool cancel = false;      // a server member whose ticket was cancelled
    int level = 0;            // index of its next level
    std::vector<i32> comp;    // original node -> its node at the current level
    slm_result *res = nullptr;
    // a server member keeps its CSR until it joins the union
    std::vector<i64> rp;
    std::vector<i32> col, w;
};

struct slm_graph {
    hipStream_t s = nullptr;
    int device = 0;
    i64 n0 = 0, nnz0 = 0, m2 = 0;
    i64 *rp0 = nullptr;
    int2 *e0 = nullptr;
    i64 *rpL[2] = {nullptr, nullptr};
    int2 *eL[2] = {nullptr, nullptr};
    int cur = -1;  // -1: level 0 arrays, else rpL[cur] / eL[cur]
    int level = 0;
    i64 n = 0, nnz = 0;
    Bins bins;
    i64 *hub_span_h = nullptr;
    Work W;
    i32 *composed = nullptr;
    bool timing = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double sweep_ms = 0;
    i64 sweeps = 0, entries = 0, bytes = 0;
    DevMem dm;  // every device buffer of the handle (dm.held: bytes held)

    // Null model (Sec. 2.2-2.4): the kind, its rational parameter num/den, and
    // the scale A of the edge term of every gain (A = M2 for the default
    // model).  W.k holds the model's node strength x; for the Erdos-Renyi
    // model it is carried from level to level by community totals (xcarry).
    int mkind = SLM_MODEL_CONFIG;
    i64 mnum = 1, mden = 1;
    i64 keyA = 0;
    i32 *xcarry = nullptr;
    // directed model: y = num * (k_out - k_in) of the input at level 0 (y0),
    // carried by community totals to the next level (ycarry); W.y holds the
    // current level's
    i32 *y0 = nullptr, *ycarry = nullptr;
    std::vector<std::pair<void *, size_t>> allocs;  // fixed buffers, freed at destroy
    bool no_fanout = false;  // keep every sweep bin on the handle's stream

    // A union handle (a batch, or a lane of a server) holds G independent
    // graphs ("members") as one disjoint union; G = 0 for a plain graph.
    // The member at position q owns the nodes [base[q], base[q+1]) of the
    // current level.  Members leave when they finish and, in a server, join
    // at level boundaries; positions are renumbered in order.
    bool is_union = false;
    int G = 0, P_cap = 0;
    std::vector<Member> mem;
    std::vector<i64> base;
    std::vector<Member> mem0;  // a batch's members at level 0 (for every run)
    std::vector<i64> base0;
    i32 *gidL[3] = {nullptr, nullptr, nullptr};  // per node: position ([2] = level 0)
    i32 *m2nL[3] = {nullptr, nullptr, nullptr};  // per node: M2 of its graph
    i64 *d_gbase = nullptr, *d_first = nullptr, *d_gcb = nullptr, *d_accI = nullptr,
        *d_accS = nullptr, *d_shift = nullptr, *d_gvalid = nullptr, *d_m2p = nullptr;
    u64 *d_gseed = nullptr;
    i32 *d_glev = nullptr, *d_newpos = nullptr;
    i32 *lab2 = nullptr;
    // shrinking a union within a level to the graphs that still move
    SubMember *d_sub = nullptr;
    SaveMember *d_save = nullptr;
    i64 *d_lbn = nullptr, *d_rpb = nullptr;
    i64 shrink_min = (i64)1 << 16;  // fewest union nodes worth a shrink (< 0: never)
};

// ------------------------------------------------------------------ helpers
void *DevMem::get(size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (fn_alloc) {
        p = fn_alloc(ctx, bytes, (void *)s);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (!p)
        throw SlmError{SLM_E_NOMEM, "device allocation of " + std::to_string(bytes) +
                                        " bytes failed"};
    held += (i64)bytes;
    return p;
}

void DevMem::put(void *p, size_t bytes)
{
    if (!p) return;
    if (bytes == 0) bytes = 256;
    if (fn_free) fn_free(ctx, p, (void *)s);
    else (void)hipFree(p);
    held -= (i64)bytes;
}

// A buffer the handle keeps until it is destroyed.
template <typename T>
static T *dalloc(slm_graph *g, i64 count)
{
    if (count < 1) count = 1;
    const size_t bytes = sizeof(T) * (size_t)count;
    g->allocs.reserve(g->allocs.size() + 1);
    void *p = g->dm.get(bytes);
    g->allocs.push_back({p, bytes});
    return (T *)p;
}

// Takes the allocator of a create call (null: hipMalloc / hipFree).
static void set_allocator(slm_graph *g, const slm_allocator *a)
{
    if (!a) return;
    if (!a->alloc || !a->free)
        throw SlmError{SLM_E_INVALID, "an allocator needs both alloc and free"};
    g->dm.ctx = a->ctx;
    g->dm.fn_alloc = a->alloc;
    g->dm.fn_free = a->free;
}

static LevelView view(slm_graph *g)
{
    LevelView L;
    L.rp = g->cur < 0 ? g->rp0 : g->rpL[g->cur];
    L.e = g->cur < 0 ? g->e0 : g->eL[g->cur];
    L.k = g->W.k;
    L.diag = g->W.diag;
    L.n = g->n;
    L.nnz = g->nnz;
    L.m2 = g->keyA;
    L.y = g->mkind == SLM_MODEL_DIRECTED ? g->W.y : nullptr;
    L.sy = g->mkind == SLM_MODEL_DIRECTED ? g->W.sigy : nullptr;
    L.m2n = nullptr;
    L.gid = nullptr;
    L.gbase = nullptr;
    L.gseed = nullptr;
    L.glev = nullptr;
    if (g->is_union) {
        const int c = g->cur < 0 ? 2 : g->cur;
        L.m2n = g->m2nL[c];
        L.gid = g->gidL[c];
        L.gbase = g->d_gbase;
        L.gseed = g->d_gseed;
        L.glev = g->d_glev;
    }
    return L;
}

// Device buffers that only grow.
template <typename T>
static void grow_buf(slm_graph *g, T *&p, i64 &cap, i64 need)
{
    dm_grow(g->dm, p, cap, need, 64);
}

static void release_bins(slm_graph *g)
{
    Bins &B = g->bins;
    DevMem &dm = g->dm;
    dm.put(B.chunk_hub, sizeof(i32) * B.cap_chunk_hub);
    dm.put(B.chunk_beg, sizeof(i64) * B.cap_chunk_beg);
    dm.put(B.hchunk, sizeof(HubChunk) * B.cap_hchunk);
    dm.put(B.chunk_off_of_hub, sizeof(i32) * B.cap_chunk_off);
    dm.put(B.htile, sizeof(HubTile) * B.cap_htile);
    dm.put(B.tile_off_of_hub, sizeof(i32) * B.cap_tile_off);
    dm.put(B.span, sizeof(i64) * B.cap_span);
    const int cap = B.hub_cap, tbits = B.hub_tbits;
    i32 grid[NBINS];
    for (int b = 0; b < NBINS; b++) grid[b] = B.grid_cap[b];
    B = Bins();
    B.hub_cap = cap;
    B.hub_tbits = tbits;
    for (int b = 0; b < NBINS; b++) B.grid_cap[b] = grid[b];
}

// Bounds of a null model other than the default: every gain within 2^62
// (A * M2 and (sum of x)^2 at most 2^61).
static void check_model_bounds(slm_graph *g)
{
    const i64 B61 = (i64)1 << 61;
    REQUIRE(g->m2 < ((i64)1 << 31), SLM_E_OVERFLOW, "total weight M2 must be below 2^31");
    if (g->mkind == SLM_MODEL_CONFIG && g->mnum == 1 && g->mden == 1) return;
    const i64 xt_unit = g->mkind == SLM_MODEL_ER ? g->n0 : g->m2;  // sum of x / num
    REQUIRE(g->mnum <= ((i64)1 << 30) && (xt_unit == 0 || g->mnum <= ((i64)1 << 30) / xt_unit),
            SLM_E_OVERFLOW, "the model's strengths must sum to at most 2^30");
    REQUIRE(g->mnum <= B61 / g->mden, SLM_E_OVERFLOW, "num * den too large");
    const i64 nd = g->mnum * g->mden;
    const i64 base = g->mkind == SLM_MODEL_ER ? 1 : g->m2;
    REQUIRE(base == 0 || nd <= B61 / base, SLM_E_OVERFLOW, "the scale A of the gains is too large");
    REQUIRE(g->m2 == 0 || nd * base <= B61 / g->m2, SLM_E_OVERFLOW,
            "A * M2 must be at most 2^61");
}

// Degree bins, hub work lists, strengths and entry rows of the current level.
static void setup_level(slm_graph *g)
{
    hipStream_t s = g->s;
    Work &W = g->W;
    Bins &B = g->bins;
    B.nhub = 0;
    B.nchunk = 0;
    B.ntile = 0;
    B.hub_entries = 0;
    B.npoff = 0;
    const i64 n = g->n;
    const i64 *rp = g->cur < 0 ? g->rp0 : g->rpL[g->cur];
    const int2 *e = g->cur < 0 ? g->e0 : g->eL[g->cur];
    for (int b = 0; b <= NBINS; b++) B.off[b] = 0;
    if (n > 0) {
        grow_buf(g, W.bscan, W.bscan_cap, bin_scan_elems(n));
        launch_bins(rp, n, W.bscan, W.counters, B.nodes, s);
        read_scalars(W, W.counters, NBINS + 1, s);
        for (int b = 0; b <= NBINS; b++) B.off[b] = W.h_scal[b];
        launch_rowdesc(B.nodes, rp, n, B.rowd, s);
        const i64 nhub = B.off[BIN_HUB + 1] - B.off[BIN_HUB];
        B.nhub = (i32)nhub;
        B.hub_node = B.nodes + B.off[BIN_HUB];
        if (nhub > 0) {
            grow_buf(g, B.span, B.cap_span, 2 * nhub);
            launch_hub_degrees(rp, B.hub_node, (i32)nhub, B.span, s);
            std::vector<i64> span(2 * nhub);
            HIPCHK(hipMemcpyAsync(span.data(), B.span, sizeof(i64) * 2 * nhub,
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            std::vector<i32> hnode(nhub);
            HIPCHK(hipMemcpyAsync(hnode.data(), B.hub_node, sizeof(i32) * nhub,
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            std::vector<i32> chunk_first(nhub + 1, 0);
            std::vector<i32> chunk_hub;
            std::vector<i64> chunk_beg;
            std::vector<HubChunk> hchunk;
            std::vector<i32> tile_first(nhub + 1, 0);
            std::vector<HubTile> htile;
            i64 out = 0, pb = 0;
            for (i64 h = 0; h < nhub; h++) {
                const i64 b0 = span[2 * h], b1 = span[2 * h + 1], deg = b1 - b0;
                int lp = 0;
                while (((i64)HUB_PART << lp) < deg && (1 << lp) < HUB_PMAX) lp++;
                const i64 pb0 = pb;
                chunk_first[h] = (i32)chunk_hub.size();
                for (i64 c = b0; c < b1; c += HUB_CHUNK) {
                    chunk_hub.push_back((i32)h);
                    chunk_beg.push_back(c);
                    HubChunk hc{};
                    hc.beg = c;
                    hc.end = c + HUB_CHUNK < b1 ? c + HUB_CHUNK : b1;
                    hc.out = out + (c - b0);
                    hc.pbase = pb;
                    hc.node = hnode[h];
                    hc.logp = lp;
                    hchunk.push_back(hc);
                    pb += ((i64)1 << lp) + 1;
                }
                tile_first[h] = (i32)htile.size();
                for (i32 q = 0; q < (1 << lp); q++) {
                    HubTile ht{};
                    ht.pbase0 = pb0;
                    ht.node = hnode[h];
                    ht.c0 = chunk_first[h];
                    ht.nch = (i32)chunk_hub.size() - chunk_first[h];
                    ht.logp = lp;
                    ht.p = q;
                    htile.push_back(ht);
                }
                out += deg;
            }
            chunk_first[nhub] = (i32)chunk_hub.size();
            tile_first[nhub] = (i32)htile.size();
            B.ntile = (i64)htile.size();
            B.nchunk = (i64)chunk_hub.size();
            B.hub_entries = out;
            B.npoff = pb;
            grow_buf(g, B.htile, B.cap_htile, B.ntile);
            grow_buf(g, B.tile_off_of_hub, B.cap_tile_off, nhub + 1);
            grow_buf(g, B.chunk_off_of_hub, B.cap_chunk_off, nhub + 1);
            grow_buf(g, B.chunk_hub, B.cap_chunk_hub, B.nchunk);
            grow_buf(g, B.chunk_beg, B.cap_chunk_beg, B.nchunk);
            grow_buf(g, B.hchunk, B.cap_hchunk, B.nchunk);
            HIPCHK(hipMemcpyAsync(B.htile, htile.data(), sizeof(HubTile) * B.ntile,
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(B.tile_off_of_hub, tile_first.data(), sizeof(i32) * (nhub + 1),
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(B.chunk_off_of_hub, chunk_first.data(), sizeof(i32) * (nhub + 1),
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(B.chunk_hub, chunk_hub.data(), sizeof(i32) * B.nchunk,
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(B.chunk_beg, chunk_beg.data(), sizeof(i64) * B.nchunk,
                                  hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(B.hchunk, hchunk.data(), sizeof(HubChunk) * B.nchunk,
                                  hipMemcpyHostToDevice, s));
            if (B.ntile > W.hub_tile_cap) {
                i64 c1 = W.hub_tile_cap, c2 = W.hub_tile_cap;
                dm_grow(g->dm, W.hub_tkey, c1, B.ntile, 64);
                dm_grow(g->dm, W.hub_tid, c2, B.ntile, 64);
                W.hub_tile_cap = c1;
            }
            grow_buf(g, W.hub_part, W.hub_part_cap, B.hub_entries);
            grow_buf(g, W.hub_poff, W.hub_poff_cap, B.npoff);
            grow_buf(g, W.hub_cwin, W.hub_cwin_cap, B.nchunk);
            if (B.nchunk > W.hub_chunk_cap) {
                i64 c1 = W.hub_chunk_cap, c2 = W.hub_chunk_cap;
                dm_grow(g->dm, W.hub_ckey, c1, B.nchunk, 64);
                dm_grow(g->dm, W.hub_cid, c2, B.nchunk, 64);
                W.hub_chunk_cap = c1;
            }
            HIPCHK(hipStreamSynchronize(s));
        }
    }
    i64 m2 = level_strengths(W, rp, e, B, n, W.k, W.diag, s);
    if (g->level == 0) {
        g->m2 = m2;
        if (!g->is_union) check_model_bounds(g);
        g->keyA = g->mkind == SLM_MODEL_ER ? g->mnum * g->mden : g->mnum * g->mden * m2;
    }
    // node strengths of the model: num times the row sums (configuration
    // model), or num times the original nodes a node stands for (Erdos-Renyi)
    if (n > 0 && (g->mkind == SLM_MODEL_CONFIG || g->mkind == SLM_MODEL_DIRECTED) &&
        g->mnum != 1)
        launch_scale_i32(W.k, (i32)g->mnum, n, s);
    if (n > 0 && g->mkind == SLM_MODEL_DIRECTED)
        HIPCHK(hipMemcpyAsync(W.y, g->level == 0 ? g->y0 : g->ycarry, sizeof(i32) * n,
                              hipMemcpyDeviceToDevice, s));
    if (n > 0 && g->mkind == SLM_MODEL_ER) {
        if (g->level == 0) launch_fill_i32(W.k, (i32)g->mnum, n, s);
        else HIPCHK(hipMemcpyAsync(W.k, g->xcarry, sizeof(i32) * n, hipMemcpyDeviceToDevice, s));
    }
    LevelView L = view(g);
    fill_src(L, B, W.src, s);
}

static void alloc_work(slm_graph *g)
{
    Work &W = g->W;
    W.dm = &g->dm;
    g->dm.s = g->s;
    const i64 n = g->n0, nnz = g->nnz0;
    W.n0 = n;
    W.nnz0 = nnz;
    int kmax = 2;
    while (((i64)1 << (kmax - 2)) < n) kmax++;
    W.kmax = kmax;
    W.a = dalloc<i32>(g, n);
    W.lab = dalloc<i32>(g, n);
    W.comp = dalloc<i32>(g, n);
    W.best_c = dalloc<i32>(g, n);
    W.w_own = dalloc<i32>(g, n);
    W.wc = dalloc<i32>(g, n);
    W.sigma = dalloc<i32>(g, n);
    W.k = dalloc<i32>(g, n);
    W.diag = dalloc<i32>(g, n);
    W.delta = dalloc<i64>(g, n);
    W.cyc = dalloc<uint8_t>(g, n);
    W.act = dalloc<uint8_t>(g, n);
    W.hasc = dalloc<uint8_t>(g, n);
    W.exam = dalloc<uint8_t>(g, n);
    W.exam_next = dalloc<uint8_t>(g, n);
    W.moved = dalloc<uint8_t>(g, n);
    W.pact = dalloc<uint8_t>(g, n);
    W.accept = dalloc<uint8_t>(g, n);
    W.head = dalloc<uint8_t>(g, n);
    W.claim = dalloc<i32>(g, n);
    W.L = dalloc<i32>(g, n);
    W.pos = dalloc<i32>(g, n);
    W.cnode = dalloc<i32>(g, n);
    W.mlist = dalloc<i32>(g, n);
    W.A0 = dalloc<i32>(g, n);
    W.A1 = dalloc<i32>(g, n);
    W.M0 = dalloc<i32>(g, n);
    W.M1 = dalloc<i32>(g, n);
    W.J = dalloc<i32>(g, (i64)kmax * (n > 0 ? n : 1));
    W.D0 = dalloc<i32>(g, n);
    W.D1 = dalloc<i32>(g, n);
    W.S0 = dalloc<i64>(g, n);
    W.S1 = dalloc<i64>(g, n);
    W.subk = dalloc<i64>(g, n);
    W.cut = dalloc<i64>(g, n);
    W.key = dalloc<i64>(g, n);
    W.bestkey = dalloc<i64>(g, n);
    W.cbest_key = dalloc<i64>(g, n);
    W.woff = dalloc<i64>(g, n);
    W.noff = dalloc<i64>(g, n);
    W.bestpair = dalloc<u64>(g, n);
    W.cbest_pair = dalloc<u64>(g, n);
    W.nca0 = dalloc<i32>(g, n);
    W.nca1 = dalloc<i32>(g, n);
    W.wbd = dalloc<i32>(g, n);
    W.ccnt = dalloc<i32>(g, n);
    W.cfill = dalloc<i32>(g, n);
    W.clist = dalloc<i32>(g, n);
    W.coff = dalloc<i64>(g, n + 1);
    W.fidx = dalloc<i32>(g, n);
    W.flist = dalloc<i32>(g, n);
    W.fcnt = dalloc<i32>(g, n);
    W.flen = dalloc<i32>(g, n);
    W.mem = dalloc<i32>(g, n);
    W.ptmp = dalloc<i32>(g, n);
    W.pord = dalloc<i32>(g, n);
    W.pchl = dalloc<i32>(g, 2 * n);
    W.plvl = dalloc<i32>(g, 2 * n + 1);
    W.part = dalloc<i32>(g, n);
    W.win = dalloc<i32>(g, n);
    W.psub = dalloc<i32>(g, n);
    W.pcut = dalloc<i32>(g, n);
    W.pdep = dalloc<i32>(g, n);
    W.proot = dalloc<i32>(g, n);
    W.chs = dalloc<i32>(g, n);
    W.chc = dalloc<i32>(g, n);
    W.mem_off = dalloc<i64>(g, n + 1);
    W.pdp = dalloc<i64>(g, 2 * n + 1);
    W.woff_f = dalloc<i64>(g, n + 1);
    W.noff_f = dalloc<i64>(g, n + 1);
    W.wsz = dalloc<i64>(g, n);
    W.nsz = dalloc<i64>(g, n);
    W.pstk = dalloc<int4>(g, n);
    W.minm = dalloc<i32>(g, n);
    W.rank = dalloc<i64>(g, n + 1);
    W.scan_tmp = dalloc<i64>(g, scan_tmp_elems(std::max(n, nnz) + 1) + 16);
    W.counters = dalloc<i64>(g, 16);
    W.stepf = dalloc<i32>(g, 64);
    W.changed = dalloc<int>(g, 4);
    W.src = dalloc<i32>(g, nnz);
    W.rk0 = dalloc<u64>(g, nnz);
    W.rk1 = dalloc<u64>(g, nnz);
    W.rv0 = dalloc<i32>(g, nnz + 1);  // + 1: the segment starts of AGGREGATE
    W.rv1 = dalloc<i32>(g, nnz + 1);
    W.cnt = dalloc<i32>(g, n);
    W.roff = dalloc<i64>(g, n + 1);
    W.head_e = dalloc<uint8_t>(g, nnz);
    W.rank_e = dalloc<i64>(g, nnz + 1);
    g->bins.nodes = dalloc<i32>(g, n);
    g->bins.rowd = dalloc<int4>(g, n);
    g->bins.ls = dalloc<int2>(g, n);
    g->composed = dalloc<i32>(g, n);
    g->rpL[0] = dalloc<i64>(g, n + 1);
    g->rpL[1] = dalloc<i64>(g, n + 1);
    g->eL[0] = dalloc<int2>(g, nnz);
    g->eL[1] = dalloc<int2>(g, nnz);
    void *hs = nullptr;
    HIPCHK(hipHostMalloc(&hs, sizeof(i64) * 64, hipHostMallocDefault));
    W.h_scal = (i64 *)hs;
    // Side streams for the sweep of large levels.  A server lane has none:
    // its streams would share the device's few hardware queues with the other
    // lanes and wait behind their long kernels.  SLM_SERIAL_SWEEP=1 keeps
    // every bin on the handle's stream (per-kernel timing without overlap).
    if (!g->no_fanout && !getenv("SLM_SERIAL_SWEEP")) {
        HIPCHK(hipEventCreateWithFlags(&W.fan.fork, hipEventDisableTiming));
        for (int q = 0; q < FAN_SIDE; q++) {
            HIPCHK(hipStreamCreateWithFlags(&W.fan.side[q], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&W.fan.join[q], hipEventDisableTiming));
        }
    }
}

static slm_status fail(const SlmError &e)
{
    g_err = e.msg;
    return (slm_status)e.status;
}

#define API_BEGIN try {
#define API_END                                                                       \
    }                                                                                 \
    catch (const SlmError &e_) { return fail(e_); }                                   \
    catch (const std::bad_alloc &) { return fail(SlmError{SLM_E_NOMEM, "host allocation failed"}); } \
    return SLM_OK;


// ------------------------------------------------------------------ validation
static void validate_host(i64 n, i64 nnz, const std::vector<i64> &rp, const i32 *col,
                          const i32 *w, i64 *m2_out, bool symmetric = true)
{
    REQUIRE(rp[0] == 0 && rp[n] == nnz, SLM_E_INVALID, "row_ptr must start at 0 and end at nnz");
    i64 m2 = 0;
    for (i64 i = 0; i < n; i++) {
        REQUIRE(rp[i + 1] >= rp[i], SLM_E_INVALID, "row_ptr is not monotone");
        for (i64 e = rp[i]; e < rp[i + 1]; e++) {
            REQUIRE(col[e] >= 0 && col[e] < n, SLM_E_INVALID, "column out of range");
            REQUIRE(w[e] >= 1, SLM_E_INVALID, "weights must be positive");
            if (e > rp[i]) REQUIRE(col[e] > col[e - 1], SLM_E_INVALID,
                                   "columns must be strictly ascending in every row");
            m2 += w[e];
        }
    }
    for (i64 i = 0; i < n && symmetric; i++) {
        for (i64 e = rp[i]; e < rp[i + 1]; e++) {
            const i32 j = col[e];
            const i32 *b = col + rp[j], *en = col + rp[j + 1];
            const i32 *f = std::lower_bound(b, en, (i32)i);
            REQUIRE(f != en && *f == (i32)i && w[rp[j] + (f - b)] == w[e], SLM_E_INVALID,
                    "the matrix is not symmetric");
        }
    }
    *m2_out = m2;
}

__global__ void k_pack_edges(const i32 *__restrict__ col, const i32 *__restrict__ w, i64 nnz,
                             int2 *__restrict__ e)
{
    for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j < nnz;
         j += (i64)gridDim.x * blockDim.x)
        e[j] = make_int2(col[j], w[j]);
}

__global__ void k_widen_rp(const i32 *__restrict__ rp32, i64 n1, i64 *__restrict__ rp)
{
    for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j < n1;
         j += (i64)gridDim.x * blockDim.x)
        rp[j] = rp32[j];
}

__global__ void k_label_range(const i32 *__restrict__ lab, i64 n, i64 nc, int *__restrict__ bad)
{
    for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (i64)gridDim.x * blockDim.x)
        if (lab[j] < 0 || lab[j] >= nc) *bad = 1;
}

static unsigned small_grid(i64 n)
{
    i64 g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return (unsigned)g;
}

static void check_labels(slm_graph *g, const i32 *lab, i64 nc)
{
    REQUIRE(lab != nullptr || g->n == 0, SLM_E_INVALID, "null label array");
    REQUIRE(nc >= 0 && nc <= g->n, SLM_E_INVALID, "community count out of range");
    if (g->n == 0) return;
    HIPCHK(hipMemsetAsync(g->W.changed, 0, sizeof(int), g->s));
    k_label_range<<<small_grid(g->n), 256, 0, g->s>>>(lab, g->n, nc, g->W.changed);
    HIPCHK(hipMemcpyAsync(g->W.h_scal, g->W.changed, sizeof(int), hipMemcpyDeviceToHost, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    REQUIRE(*(int *)g->W.h_scal == 0, SLM_E_INVALID, "label out of range");
}

// ------------------------------------------------------------------ level loop
static void level_start(slm_graph *g, i64 *nc)
{
    Work &W = g->W;
    LevelView L = view(g);
    run_assign(L, g->bins, W.a, W.hub_ckey, W.hub_cid, g->s);
    components(W, W.a, g->n, false, g->s);
    positive(W, L, g->bins, nc, g->s);
}

// One MAXIMAL round then POSITIVE; W.lab / *nc must describe W.a.  Returns
// the valid count.
static i64 level_round(slm_graph *g, const slm_params *p, int level, int round, i64 *nc,
                       i64 *stats4, unsigned long long *gvalid = nullptr)
{
    Work &W = g->W;
    LevelView L = view(g);
    float ms = 0;
    i64 st[3] = {0, 0, 0};
    i64 valid = maximal_moves(W, L, g->bins, *nc, p->seed, level, round, p->accept_p, st, g->s,
                              g->timing, g->ev0, g->ev1, &ms, gvalid);
    if (g->timing) {
        g->sweep_ms += ms;
        g->sweeps++;
        g->entries += g->nnz;
        g->bytes += 8 * g->nnz + 32 * g->n + 4 * (*nc);
    }
    i64 splits = 0;
    if (valid > 0) {
        components(W, W.a, g->n, false, g->s);
        mark_changed_communities(W, g->n, g->s);
        splits = positive(W, L, g->bins, nc, g->s, W.pact);
    }
    if (stats4) {
        stats4[0] = st[0];
        stats4[1] = st[1];
        stats4[2] = st[2];
        stats4[3] = splits;
    }
    return valid;
}

static void run_level(slm_graph *g, const slm_params *p, int level, i64 *nc, int32_t *rounds,
                      int32_t *conv)
{
    level_start(g, nc);
    int r = 0;
    *conv = 0;
    while (r < p->max_rounds) {
        i64 valid = level_round(g, p, level, r, nc, nullptr);
        if (valid == 0) {
            *conv = 1;
            break;
        }
        r++;
    }
    *rounds = r;
}

// AGGREGATE into the other level buffer; the caller runs setup_level.
static void contract_only(slm_graph *g, const i32 *lab, i64 nc)
{
    REQUIRE(nc < g->n, SLM_E_STATE, "contraction needs fewer communities than nodes");
    Work &W = g->W;
    LevelView L = view(g);
    const int dst = g->cur < 0 ? 0 : 1 - g->cur;
    i64 nnz2 = contract_level(W, L, g->bins, lab, nc, g->rpL[dst], g->eL[dst], g->s);
    g->cur = dst;
    g->n = nc;
    g->nnz = nnz2;
    g->level++;
}

static void do_contract(slm_graph *g, const i32 *lab, i64 nc)
{
    if ((g->mkind == SLM_MODEL_ER || g->mkind == SLM_MODEL_DIRECTED) && nc < g->n) {
        // a community's strengths at the next level are the sums over its
        // members (x for Erdos-Renyi; y for the directed model, whose x is
        // num times the row sums again)
        community_totals(g->W, view(g), lab, nc, g->s);
        if (g->mkind == SLM_MODEL_ER)
            HIPCHK(hipMemcpyAsync(g->xcarry, g->W.sigma, sizeof(i32) * nc,
                                  hipMemcpyDeviceToDevice, g->s));
        else
            HIPCHK(hipMemcpyAsync(g->ycarry, g->W.sigy, sizeof(i32) * nc,
                                  hipMemcpyDeviceToDevice, g->s));
    }
    contract_only(g, lab, nc);
    setup_level(g);
}

// Per-position device arrays of a union from the host members.
static void union_upload(slm_graph *g)
{
    const int G = g->G;
    std::vector<u64> sd(G);
    std::vector<i32> lv(G);
    std::vector<i64> m2(G);
    for (int q = 0; q < G; q++) {
        sd[q] = g->mem[q].seed;
        lv[q] = g->mem[q].level;
        m2[q] = g->mem[q].m2;
    }
    hipStream_t s = g->s;
    HIPCHK(hipMemcpyAsync(g->d_gbase, g->base.data(), sizeof(i64) * (G + 1), hipMemcpyHostToDevice, s));
    if (G > 0) {
        HIPCHK(hipMemcpyAsync(g->d_gseed, sd.data(), sizeof(u64) * G, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(g->d_glev, lv.data(), sizeof(i32) * G, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(g->d_m2p, m2.data(), sizeof(i64) * G, hipMemcpyHostToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));  // the host vectors may change right after
}

static void do_reset(slm_graph *g)
{
    if (g->is_union && !g->mem0.empty()) {
        g->mem = g->mem0;
        g->base = g->base0;
        g->G = (int)g->mem.size();
        union_upload(g);
    }
    if (g->cur < 0 && g->level == 0) return;
    g->cur = -1;
    g->level = 0;
    g->n = g->n0;
    g->nnz = g->nnz0;
    setup_level(g);
}

// Draw parameters of the single-step calls on a batch: every graph uses the
// caller's seed and level, as a run of that graph alone would.
static void batch_set_draws(slm_graph *g, u64 seed, int level)
{
    if (!g->is_union || g->G == 0) return;
    for (Member &m : g->mem) {
        m.seed = seed;
        m.level = level;
    }
    union_upload(g);
}

// ------------------------------------------------------------------ unions
static void alloc_union(slm_graph *g, int P_cap)
{
    const i64 n = g->n0;
    g->is_union = true;
    g->P_cap = P_cap;
    for (int c = 0; c < 3; c++) {
        g->gidL[c] = dalloc<i32>(g, n);
        g->m2nL[c] = dalloc<i32>(g, n);
    }
    g->lab2 = dalloc<i32>(g, n);
    g->d_gbase = dalloc<i64>(g, P_cap + 1);
    g->d_gcb = dalloc<i64>(g, P_cap + 1);
    g->d_first = dalloc<i64>(g, P_cap);
    g->d_accI = dalloc<i64>(g, P_cap);
    g->d_accS = dalloc<i64>(g, P_cap);
    g->d_shift = dalloc<i64>(g, P_cap);
    g->d_gvalid = dalloc<i64>(g, P_cap);
    g->d_m2p = dalloc<i64>(g, P_cap);
    g->d_gseed = dalloc<u64>(g, P_cap);
    g->d_glev = dalloc<i32>(g, P_cap);
    g->d_newpos = dalloc<i32>(g, P_cap);
    g->d_sub = dalloc<SubMember>(g, P_cap + 1);
    g->d_save = dalloc<SaveMember>(g, P_cap);
    g->d_lbn = dalloc<i64>(g, P_cap + 1);
    g->d_rpb = dalloc<i64>(g, P_cap + 1);
}

// Per-node position and M2 of the members at positions [p0, G).
static void union_meta(slm_graph *g, int p0, i32 *gid, i32 *m2n)
{
    i64 maxn = 0;
    for (int q = p0; q < g->G; q++) maxn = std::max(maxn, g->base[q + 1] - g->base[q]);
    batch_meta(g->d_gbase, p0, g->G - p0, g->d_m2p, maxn, gid, m2n, g->s);
}

template <typename T>
static void to_host(std::vector<T> &h, const T *d, i64 count, hipStream_t s)
{
    h.resize((size_t)count);
    if (count > 0)
        HIPCHK(hipMemcpyAsync(h.data(), d, sizeof(T) * count, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

// Appends members (with their level-0 CSRs) after the nodes of the current
// level buffer; the caller runs setup_level.  Capacity is checked by the
// caller.
static void union_append(slm_graph *g, std::vector<Member> &add)
{
    if (add.empty()) return;
    hipStream_t s = g->s;
    if (g->cur < 0) g->cur = 0;  // a server union lives in the level buffers
    i64 n_add = 0, e_add = 0;
    for (const Member &m : add) {
        n_add += m.n0;
        e_add += m.nnz0;
    }
    std::vector<i64> rp_h(n_add + 1);
    std::vector<int2> e_h(e_add);
    i64 nb = g->n, eb = g->nnz, vi = 0, ej = 0;
    const int p0 = g->G;
    for (Member &m : add) {
        for (i64 v = 0; v < m.n0; v++) rp_h[vi + v] = eb + ej + m.rp[v];
        const i32 off = (i32)(nb + vi);
        for (i64 j = 0; j < m.nnz0; j++) e_h[ej + j] = make_int2(m.col[j] + off, m.w[j]);
        g->base.push_back(nb + vi + m.n0);
        vi += m.n0;
        ej += m.nnz0;
        m.rp.clear();
        m.rp.shrink_to_fit();
        m.col.clear();
        m.col.shrink_to_fit();
        m.w.clear();
        m.w.shrink_to_fit();
        g->mem.push_back(std::move(m));
    }
    rp_h[n_add] = eb + e_add;
    add.clear();
    i64 *rp = g->rpL[g->cur];
    int2 *e = g->eL[g->cur];
    HIPCHK(hipMemcpyAsync(rp + nb, rp_h.data(), sizeof(i64) * (n_add + 1), hipMemcpyHostToDevice, s));
    if (e_add)
        HIPCHK(hipMemcpyAsync(e + eb, e_h.data(), sizeof(int2) * e_add, hipMemcpyHostToDevice, s));
    g->G = (int)g->mem.size();
    g->n = nb + n_add;
    g->nnz = eb + e_add;
    union_upload(g);  // also waits for the copies above
    union_meta(g, p0, g->gidL[g->cur], g->m2nL[g->cur]);
}

// ------------------------------------------------------- shrinking a union
// A member whose round finds no valid move keeps its state for the rest of
// the level (nothing is accepted, so the next round sees the same labels and
// finds no valid move again).  Once such members hold most of the union's
// nodes, the level goes on in a union of the others: their CSR and round
// state (assignment, labels, cycle marks) are gathered into a free level
// buffer, with every node, entry and label range shifted by its member's new
// base, so local node numbers, draws and the order of labels within a member
// are those of the full union.  At the end of the level every member's labels
// are put back in the full union's numbering.
struct UnionCut {
    bool on = false;
    int full_cur = 0;
    i64 full_n = 0, full_nnz = 0;
    std::vector<int> fpos;   // position in the current union -> in the full one
    std::vector<i64> ubase;  // node ranges of the current union's members
    std::vector<i64> ncq;    // per full position: its communities, once saved
};

// First label of every member of the current union (labels are canonical, so
// a member's are contiguous and start at its first node's), and nc at the end.
static std::vector<i64> union_label_bases(slm_graph *g, int Gc, i64 nc)
{
    std::vector<i64> first;
    batch_first_labels(g->W.lab, g->d_gbase, Gc, g->d_first, g->s);
    to_host(first, g->d_first, Gc, g->s);
    std::vector<i64> gcb(Gc + 1);
    gcb[Gc] = nc;
    for (int q = Gc - 1; q >= 0; q--) gcb[q] = first[q] >= 0 ? first[q] : gcb[q + 1];
    return gcb;
}

// Every member's labels, less its first label, into g->lab2 at the nodes'
// ids in the full union, and its community count into cut.ncq.
static void union_save(slm_graph *g, UnionCut &cut, const std::vector<i64> &gcb)
{
    const int Gc = (int)cut.fpos.size();
    std::vector<SaveMember> sv(Gc);
    for (int q = 0; q < Gc; q++) {
        sv[q] = SaveMember{cut.ubase[q], gcb[q], g->base[cut.fpos[q]]};
        cut.ncq[cut.fpos[q]] = gcb[q + 1] - gcb[q];
    }
    hipStream_t s = g->s;
    HIPCHK(hipMemcpyAsync(g->d_save, sv.data(), sizeof(SaveMember) * Gc, hipMemcpyHostToDevice, s));
    const int c = g->cur < 0 ? 2 : g->cur;
    batch_sub_save(g->gidL[c], g->n, g->W.lab, g->d_save, g->lab2, s);
    HIPCHK(hipStreamSynchronize(s));  // sv is freed on return
}

// The current union shrinks to the members with moving[q] set, into level
// buffer `target`; *nc becomes the shrunk union's community count.
static void union_shrink(slm_graph *g, UnionCut &cut, const std::vector<char> &moving, int target,
                         i64 *nc)
{
    hipStream_t s = g->s;
    Work &W = g->W;
    const int Gc = (int)cut.fpos.size();
    if (!cut.on) {
        cut.on = true;
        cut.full_cur = g->cur;
        cut.full_n = g->n;
        cut.full_nnz = g->nnz;
        cut.ncq.assign(g->G, 0);
    }
    const std::vector<i64> gcb = union_label_bases(g, Gc, *nc);
    union_save(g, cut, gcb);
    const i64 *rp_u = g->cur < 0 ? g->rp0 : g->rpL[g->cur];
    const int2 *e_u = g->cur < 0 ? g->e0 : g->eL[g->cur];
    std::vector<i64> erb;
    batch_member_rows(rp_u, g->d_gbase, Gc, g->d_rpb, s);
    to_host(erb, g->d_rpb, Gc + 1, s);
    std::vector<SubMember> sm;
    std::vector<int> fpos2;
    std::vector<i64> base2(1, 0), m2;
    std::vector<u64> sd;
    std::vector<i32> lv;
    i64 nn = 0, ne = 0, nl = 0, maxn = 0;
    for (int q = 0; q < Gc; q++) {
        if (!moving[q]) continue;
        const i64 dn = cut.ubase[q + 1] - cut.ubase[q];
        sm.push_back(SubMember{nn, ne, nl, cut.ubase[q], erb[q], gcb[q]});
        nn += dn;
        ne += erb[q + 1] - erb[q];
        nl += gcb[q + 1] - gcb[q];
        maxn = std::max(maxn, dn);
        fpos2.push_back(cut.fpos[q]);
        base2.push_back(nn);
        const Member &m = g->mem[cut.fpos[q]];
        sd.push_back(m.seed);
        lv.push_back(m.level);
        m2.push_back(m.m2);
    }
    sm.push_back(SubMember{nn, ne, nl, 0, 0, 0});
    const int G2 = (int)fpos2.size();
    HIPCHK(hipMemcpyAsync(g->d_sub, sm.data(), sizeof(SubMember) * (G2 + 1), hipMemcpyHostToDevice, s));
    batch_sub_gather(g->d_sub, G2, nn, ne, rp_u, e_u, W.a, W.lab, W.cyc, g->rpL[target],
                     g->eL[target], W.A0, W.A1, W.exam, s);
    HIPCHK(hipMemcpyAsync(W.a, W.A0, sizeof(i32) * nn, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(W.lab, W.A1, sizeof(i32) * nn, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(W.cyc, W.exam, nn, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(g->d_gbase, base2.data(), sizeof(i64) * (G2 + 1), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g->d_gseed, sd.data(), sizeof(u64) * G2, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g->d_glev, lv.data(), sizeof(i32) * G2, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g->d_m2p, m2.data(), sizeof(i64) * G2, hipMemcpyHostToDevice, s));
    batch_meta(g->d_gbase, 0, G2, g->d_m2p, maxn, g->gidL[target], g->m2nL[target], s);
    HIPCHK(hipStreamSynchronize(s));  // the host vectors are freed on return
    g->cur = target;
    g->n = nn;
    g->nnz = ne;
    setup_level(g);
    cut.fpos = std::move(fpos2);
    cut.ubase = std::move(base2);
    *nc = nl;
}

// After a round: shrink when the members still moving hold at most half of
// the union's nodes and a level buffer is free (both while the full union is
// in the level-0 arrays, the other one otherwise, so once per level then).
static void union_maybe_shrink(slm_graph *g, UnionCut &cut, const std::vector<i32> &rounds, i64 *nc)
{
    if (g->shrink_min < 0 || g->n < g->shrink_min) return;
    const int Gc = (int)cut.fpos.size();
    std::vector<char> moving(Gc, 0);
    i64 act = 0;
    for (int q = 0; q < Gc; q++) {
        moving[q] = rounds[cut.fpos[q]] < 0;
        if (moving[q]) act += cut.ubase[q + 1] - cut.ubase[q];
    }
    if (act == 0 || 2 * act > g->n) return;
    const int full = cut.on ? cut.full_cur : g->cur;
    int target;
    if (full < 0) target = g->cur == 0 ? 1 : 0;
    else if (!cut.on) target = 1 - g->cur;
    else return;
    union_shrink(g, cut, moving, target, nc);
}

// Back to the full union, with every member's labels in its numbering.
static void union_unshrink(slm_graph *g, UnionCut &cut, i64 *nc)
{
    hipStream_t s = g->s;
    const std::vector<i64> gcb = union_label_bases(g, (int)cut.fpos.size(), *nc);
    union_save(g, cut, gcb);
    g->cur = cut.full_cur;
    g->n = cut.full_n;
    g->nnz = cut.full_nnz;
    union_upload(g);
    setup_level(g);
    std::vector<i64> lb(g->G + 1, 0);
    for (int q = 0; q < g->G; q++) lb[q + 1] = lb[q] + cut.ncq[q];
    HIPCHK(hipMemcpyAsync(g->d_lbn, lb.data(), sizeof(i64) * (g->G + 1), hipMemcpyHostToDevice, s));
    const int c = g->cur < 0 ? 2 : g->cur;
    batch_sub_restore(g->gidL[c], g->n, g->lab2, g->d_lbn, g->W.lab, s);
    HIPCHK(hipStreamSynchronize(s));
    *nc = lb[g->G];
    cut.on = false;
}

// One level of Algorithm 1 for every member of the union, all in the same
// launches.  Member q draws with its own seed and level; its keys use its own
// M2.  A member whose round finds no valid move is unchanged by the rounds
// the others still need, so its rounds and convergence are its own.  At the
// end every member reads its community range from its first node, emits its
// level (labels composed onto its original nodes, n_c, N_Q, Q, rounds,
// converged), and leaves when the partition is the identity or max_levels is
// reached; the others are contracted together (setup_level is left to the
// caller, which may append members first).  Leaving members go to `done`.
// mark_cancel (may be null) is called once the level's work is done and sets
// Member::cancel on members whose request was cancelled: they leave without
// output.
static void union_level(slm_graph *g, const slm_params *p, std::vector<Member> &done,
                        const std::function<void(std::vector<Member> &)> *mark_cancel = nullptr)
{
    const int G = g->G;
    Work &W = g->W;
    hipStream_t s = g->s;
    i64 nc;
    level_start(g, &nc);
    std::vector<i32> rounds(G, -1), conv(G, 0);
    std::vector<i64> hv, first, accI, accS;
    UnionCut cut;
    cut.fpos.resize(G);
    for (int q = 0; q < G; q++) cut.fpos[q] = q;
    cut.ubase = g->base;
    int r = 0;
    while (r < p->max_rounds) {
        const int Gc = (int)cut.fpos.size();
        launch_fill_i64(g->d_gvalid, 0, Gc, s);
        const i64 valid = level_round(g, p, 0, r, &nc, nullptr, (unsigned long long *)g->d_gvalid);
        to_host(hv, g->d_gvalid, Gc, s);
        for (int q = 0; q < Gc; q++) {
            const int f = cut.fpos[q];
            if (rounds[f] < 0 && hv[q] == 0) {
                rounds[f] = r;
                conv[f] = 1;
            }
        }
        if (valid == 0) break;
        r++;
        if (r < p->max_rounds) union_maybe_shrink(g, cut, rounds, &nc);
    }
    if (cut.on) union_unshrink(g, cut, &nc);
    for (int q = 0; q < G; q++)
        if (rounds[q] < 0) rounds[q] = r;
    batch_first_labels(W.lab, g->d_gbase, G, g->d_first, s);
    to_host(first, g->d_first, G, s);
    std::vector<i64> gcb(G + 1);
    gcb[G] = nc;
    for (int q = G - 1; q >= 0; q--) gcb[q] = first[q] >= 0 ? first[q] : gcb[q + 1];
    if (mark_cancel) (*mark_cancel)(g->mem);
    std::vector<char> emit(G, 0), leave(G, 0);
    bool any_emit = false;
    for (int q = 0; q < G; q++) {
        if (g->mem[q].cancel) leave[q] = 1;  // a cancelled request: no output
        else if (gcb[q + 1] - gcb[q] == g->base[q + 1] - g->base[q]) leave[q] = 1;  // identity
        else emit[q] = any_emit = true;
    }
    if (any_emit) {
        HIPCHK(hipMemcpyAsync(g->d_gcb, gcb.data(), sizeof(i64) * (G + 1), hipMemcpyHostToDevice, s));
        modularity_graphs(W, view(g), g->bins, W.lab, nc, G, g->d_gcb, g->d_accI, g->d_accS, s);
        to_host(accI, g->d_accI, G, s);
        to_host(accS, g->d_accS, G, s);
        std::vector<i32> lab_h;
        to_host(lab_h, W.lab, g->n, s);
        // each member composes its labels and records its level on its own
        // (members of one range per host thread when the union is large)
        auto emit_range = [&](int q0, int q1) {
            for (int q = q0; q < q1; q++) {
                if (!emit[q]) continue;
                Member &m = g->mem[q];
                const i32 *lq = lab_h.data() + g->base[q];
                const i32 c0 = (i32)gcb[q];
                for (i64 v = 0; v < m.n0; v++) m.comp[v] = lq[m.comp[v]] - c0;
                const i64 nq = m.m2 * accI[q] - accS[q];
                slm_result *R = m.res;
                R->labels.push_back(m.comp);
                R->nc.push_back(gcb[q + 1] - gcb[q]);
                R->nq.push_back(nq);
                R->q.push_back((double)nq / (double)m.m2 / (double)m.m2);
                R->rounds.push_back(rounds[q]);
                R->conv.push_back(conv[q]);
                m.level++;
                if (p->max_levels > 0 && (int)R->nc.size() >= p->max_levels) leave[q] = 1;
            }
        };
        i64 work = 0;
        for (int q = 0; q < G; q++)
            if (emit[q]) work += g->mem[q].n0;
        const int hw = (int)std::thread::hardware_concurrency();
        const int T = std::min(std::min(hw > 0 ? hw : 1, 16), G);
        if (T <= 1 || work < ((i64)1 << 20)) {
            emit_range(0, G);
        } else {
            // contiguous member ranges of about work / T original nodes each
            std::vector<int> cut_at(1, 0);
            i64 acc = 0;
            for (int q = 0; q < G && (int)cut_at.size() < T; q++) {
                if (emit[q]) acc += g->mem[q].n0;
                if (acc * T >= work * (i64)cut_at.size()) cut_at.push_back(q + 1);
            }
            cut_at.push_back(G);
            std::vector<std::thread> th;
            for (size_t r = 0; r + 1 < cut_at.size(); r++)
                if (cut_at[r] < cut_at[r + 1]) th.emplace_back(emit_range, cut_at[r], cut_at[r + 1]);
            for (std::thread &t : th) t.join();
        }
    }
    // the members that stay form the next level's union, in order
    std::vector<i64> shift(G, -1), nbase(1, 0);
    std::vector<i32> newpos(G, -1);
    std::vector<Member> stay;
    i64 gone = 0, nc2 = 0;
    for (int q = 0; q < G; q++) {
        const i64 ncq = gcb[q + 1] - gcb[q];
        if (leave[q]) {
            gone += ncq;
            done.push_back(std::move(g->mem[q]));
            continue;
        }
        shift[q] = gone;
        newpos[q] = (i32)stay.size();
        nc2 += ncq;
        nbase.push_back(nc2);
        stay.push_back(std::move(g->mem[q]));
    }
    g->level++;
    if (stay.empty()) {
        g->mem.clear();
        g->base.assign(1, 0);
        g->G = 0;
        g->n = g->nnz = 0;
        return;
    }
    HIPCHK(hipMemcpyAsync(g->d_shift, shift.data(), sizeof(i64) * G, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(g->d_newpos, newpos.data(), sizeof(i32) * G, hipMemcpyHostToDevice, s));
    const int dst = g->cur < 0 ? 0 : 1 - g->cur;
    const int src = g->cur < 0 ? 2 : g->cur;
    batch_relabel(W.lab, g->gidL[src], g->m2nL[src], g->d_shift, g->d_newpos, g->n, g->lab2,
                  g->gidL[dst], g->m2nL[dst], s);
    contract_only(g, g->lab2, nc2);
    g->mem = std::move(stay);
    g->base = std::move(nbase);
    g->G = (int)g->mem.size();
    union_upload(g);
}

// All members of a batch through Algorithm 1; results by batch index.
static void batch_run(slm_graph *g, const slm_params *p, const u64 *seeds,
                      std::vector<slm_result *> &res)
{
    do_reset(g);
    for (int q = 0; q < g->G; q++) {
        Member &m = g->mem[q];
        m.seed = seeds ? seeds[m.ticket] : p->seed;
        m.level = 0;
        m.res = res[m.ticket];
        m.res->n0 = m.n0;
        m.comp.resize(m.n0);
        for (i64 v = 0; v < m.n0; v++) m.comp[v] = (i32)v;
    }
    union_upload(g);
    std::vector<Member> done;
    while (g->G > 0 && g->n > 0) {
        union_level(g, p, done);
        if (g->G > 0) setup_level(g);
    }
    HIPCHK(hipStreamSynchronize(g->s));
}

// Device copy of a host CSR (entries already packed) and the level-0 state.
static void init_from_host(slm_graph *g, const i64 *rp_h, const int2 *e_h)
{
    alloc_work(g);
    g->rp0 = dalloc<i64>(g, g->n0 + 1);
    g->e0 = dalloc<int2>(g, g->nnz0);
    HIPCHK(hipMemcpyAsync(g->rp0, rp_h, sizeof(i64) * (g->n0 + 1), hipMemcpyHostToDevice, g->s));
    if (g->nnz0)
        HIPCHK(hipMemcpyAsync(g->e0, e_h, sizeof(int2) * g->nnz0, hipMemcpyHostToDevice, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    HIPCHK(hipEventCreate(&g->ev0));
    HIPCHK(hipEventCreate(&g->ev1));
    setup_level(g);
}

// ================================================================== ABI
extern "C" {

void slm_params_default(slm_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->seed = 0;
    p->accept_p = 1ull << 31;
    p->max_rounds = 64;
    p->max_levels = 0;
    p->validate = 1;
}

const char *slm_last_error(void)
{
    return g_err.c_str();
}

void slm_destroy(slm_graph *g)
{
    if (!g) return;
    (void)hipStreamSynchronize(g->s);
    release_bins(g);
    for (auto &pb : g->allocs) g->dm.put(pb.first, pb.second);
    Work &W = g->W;
    DevMem &dm = g->dm;
    dm.put(W.W, sizeof(i64) * W.W_cap);
    dm.put(W.hist, sizeof(i64) * 2 * W.hist_cap);
    dm.put(W.bscan, sizeof(i64) * W.bscan_cap);
    dm.put(W.hub_part, sizeof(int2) * W.hub_part_cap);
    dm.put(W.hub_poff, sizeof(i64) * W.hub_poff_cap);
    dm.put(W.hub_cwin, sizeof(i32) * W.hub_cwin_cap);
    dm.put(W.hub_ckey, sizeof(i64) * W.hub_chunk_cap);
    dm.put(W.hub_cid, sizeof(i32) * W.hub_chunk_cap);
    dm.put(W.hub_tkey, sizeof(i64) * W.hub_tile_cap);
    dm.put(W.hub_tid, sizeof(i32) * W.hub_tile_cap);
    if (W.h_scal) (void)hipHostFree(W.h_scal);
    for (int q = 0; q < FAN_SIDE; q++) {
        if (W.fan.side[q]) (void)hipStreamDestroy(W.fan.side[q]);
        if (W.fan.join[q]) (void)hipEventDestroy(W.fan.join[q]);
    }
    if (W.fan.fork) (void)hipEventDestroy(W.fan.fork);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    delete g;
}

static slm_status create_impl(int64_t n, int64_t nnz, const void *row_ptr, int row_ptr_bytes,
                              const int32_t *col, const int32_t *w, int inputs_on_device,
                              int validate, const slm_model *model, void *hip_stream,
                              const slm_allocator *alloc, slm_graph **out)
{
    slm_graph *g = nullptr;
    try {
        REQUIRE(out != nullptr, SLM_E_INVALID, "null output handle");
        *out = nullptr;
        if (model) {
            REQUIRE(model->kind == SLM_MODEL_CONFIG || model->kind == SLM_MODEL_ER ||
                        model->kind == SLM_MODEL_DIRECTED,
                    SLM_E_INVALID, "unknown null model kind");
            REQUIRE(model->num >= 1 && model->den >= 1, SLM_E_INVALID,
                    "the model parameter num/den needs num >= 1 and den >= 1");
        }
        REQUIRE(n >= 0 && nnz >= 0, SLM_E_INVALID, "negative size");
        REQUIRE(row_ptr_bytes == 4 || row_ptr_bytes == 8, SLM_E_INVALID, "row_ptr_bytes must be 4 or 8");
        REQUIRE(row_ptr != nullptr, SLM_E_INVALID, "null row_ptr");
        REQUIRE(nnz == 0 || (col && w), SLM_E_INVALID, "null col or w");
        REQUIRE(n < ((i64)1 << 31) - 1, SLM_E_OVERFLOW, "n must be below 2^31 - 1");
        REQUIRE(nnz < ((i64)1 << 40), SLM_E_OVERFLOW, "too many entries");
        g = new slm_graph();
        g->s = (hipStream_t)hip_stream;
        if (model) {
            g->mkind = model->kind;
            g->mnum = model->num;
            g->mden = model->den;
        }
        set_allocator(g, alloc);
        HIPCHK(hipGetDevice(&g->device));
        g->n0 = g->n = n;
        g->nnz0 = g->nnz = nnz;
        // host copies for validation (or the inputs themselves when on host)
        std::vector<i64> rp_h;
        std::vector<i32> col_h, w_h;
        const i32 *colp = col, *wp = w;
        i64 m2 = -1;
        if (!inputs_on_device || validate) {
            rp_h.resize(n + 1);
            if (inputs_on_device) {
                std::vector<char> tmp((size_t)(n + 1) * row_ptr_bytes);
                HIPCHK(hipMemcpy(tmp.data(), row_ptr, tmp.size(), hipMemcpyDeviceToHost));
                for (i64 i = 0; i <= n; i++)
                    rp_h[i] = row_ptr_bytes == 8 ? ((const i64 *)tmp.data())[i]
                                                 : ((const i32 *)tmp.data())[i];
                col_h.resize(nnz);
                w_h.resize(nnz);
                if (nnz) {
                    HIPCHK(hipMemcpy(col_h.data(), col, sizeof(i32) * nnz, hipMemcpyDeviceToHost));
                    HIPCHK(hipMemcpy(w_h.data(), w, sizeof(i32) * nnz, hipMemcpyDeviceToHost));
                }
                colp = col_h.data();
                wp = w_h.data();
            } else {
                for (i64 i = 0; i <= n; i++)
                    rp_h[i] = row_ptr_bytes == 8 ? ((const i64 *)row_ptr)[i]
                                                 : ((const i32 *)row_ptr)[i];
            }
            if (validate) {
                validate_host(n, nnz, rp_h, colp, wp, &m2, g->mkind != SLM_MODEL_DIRECTED);
                if (g->mkind == SLM_MODEL_DIRECTED) m2 *= 2;  // the sum of W + W^T
                REQUIRE(m2 < ((i64)1 << 31), SLM_E_OVERFLOW, "total weight M2 must be below 2^31");
            } else {
                REQUIRE(rp_h[0] == 0 && rp_h[n] == nnz, SLM_E_INVALID, "row_ptr must start at 0 and end at nnz");
            }
        }
        // the directed model runs on S = W + W^T: room for up to 2 nnz entries
        if (g->mkind == SLM_MODEL_DIRECTED) g->nnz0 = g->nnz = 2 * nnz;
        alloc_work(g);
        g->rp0 = dalloc<i64>(g, n + 1);
        g->e0 = dalloc<int2>(g, g->nnz0);
        if (g->mkind == SLM_MODEL_ER) g->xcarry = dalloc<i32>(g, n);
        if (g->mkind == SLM_MODEL_DIRECTED) {
            g->y0 = dalloc<i32>(g, n);
            g->ycarry = dalloc<i32>(g, n);
            g->W.y = dalloc<i32>(g, n);
            g->W.sigy = dalloc<i32>(g, n);
            g->W.suby = dalloc<i64>(g, n);
        }
        if (!inputs_on_device) {
            HIPCHK(hipMemcpyAsync(g->rp0, rp_h.data(), sizeof(i64) * (n + 1), hipMemcpyHostToDevice, g->s));
            if (nnz) {
                std::vector<int2> e_h(nnz);
                for (i64 j = 0; j < nnz; j++) e_h[j] = make_int2(colp[j], wp[j]);
                HIPCHK(hipMemcpyAsync(g->e0, e_h.data(), sizeof(int2) * nnz, hipMemcpyHostToDevice, g->s));
                HIPCHK(hipStreamSynchronize(g->s));
            }
        } else {
            if (row_ptr_bytes == 8)
                HIPCHK(hipMemcpyAsync(g->rp0, row_ptr, sizeof(i64) * (n + 1), hipMemcpyDeviceToDevice, g->s));
            else
                k_widen_rp<<<small_grid(n + 1), 256, 0, g->s>>>((const i32 *)row_ptr, n + 1, g->rp0);
            if (nnz) k_pack_edges<<<small_grid(nnz), 256, 0, g->s>>>(col, w, nnz, g->e0);
        }
        HIPCHK(hipEventCreate(&g->ev0));
        HIPCHK(hipEventCreate(&g->ev1));
        if (g->mkind == SLM_MODEL_DIRECTED) {
            // y0 = num (k_out - k_in) of W, then the level-0 matrix becomes S
            const i64 nnz_s = symmetrize_level(g->W, g->rp0, g->e0, n, nnz, g->y0, g->s);
            if (g->mnum != 1) launch_scale_i32(g->y0, (i32)g->mnum, n, g->s);
            g->nnz0 = g->nnz = nnz_s;
        }
        setup_level(g);
        REQUIRE(g->m2 < ((i64)1 << 31), SLM_E_OVERFLOW, "total weight M2 must be below 2^31");
        *out = g;
        return SLM_OK;
    } catch (const SlmError &e) {
        if (g) slm_destroy(g);
        return fail(e);
    } catch (const std::bad_alloc &) {
        if (g) slm_destroy(g);
        return fail(SlmError{SLM_E_NOMEM, "host allocation failed"});
    }
}

slm_status slm_create(int64_t n, int64_t nnz, const void *row_ptr, int row_ptr_bytes,
                      const int32_t *col, const int32_t *w, int inputs_on_device, int validate,
                      void *hip_stream, const slm_allocator *alloc, slm_graph **out)
{
    return create_impl(n, nnz, row_ptr, row_ptr_bytes, col, w, inputs_on_device, validate,
                       nullptr, hip_stream, alloc, out);
}

slm_status slm_create_model(int64_t n, int64_t nnz, const void *row_ptr, int row_ptr_bytes,
                            const int32_t *col, const int32_t *w, int inputs_on_device,
                            int validate, const slm_model *model, void *hip_stream,
                            const slm_allocator *alloc, slm_graph **out)
{
    return create_impl(n, nnz, row_ptr, row_ptr_bytes, col, w, inputs_on_device, validate,
                       model, hip_stream, alloc, out);
}

slm_status slm_level_info(const slm_graph *g, int32_t *level, int64_t *n_t, int64_t *nnz_t,
                          int64_t *m2)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    if (level) *level = g->level;
    if (n_t) *n_t = g->n;
    if (nnz_t) *nnz_t = g->nnz;
    if (m2) *m2 = g->m2;
    API_END
}

slm_status slm_reset(slm_graph *g)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    do_reset(g);
    API_END
}

slm_status slm_export_level(slm_graph *g, int64_t *row_ptr, int32_t *col, int32_t *w)
{
    API_BEGIN
    REQUIRE(g != nullptr && row_ptr != nullptr, SLM_E_INVALID, "null argument");
    REQUIRE(g->nnz == 0 || (col && w), SLM_E_INVALID, "null col or w");
    LevelView L = view(g);
    HIPCHK(hipMemcpyAsync(row_ptr, L.rp, sizeof(i64) * (g->n + 1), hipMemcpyDeviceToHost, g->s));
    std::vector<int2> e_h(g->nnz);
    if (g->nnz)
        HIPCHK(hipMemcpyAsync(e_h.data(), L.e, sizeof(int2) * g->nnz, hipMemcpyDeviceToHost, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    for (i64 j = 0; j < g->nnz; j++) {
        col[j] = e_h[j].x;
        w[j] = e_h[j].y;
    }
    API_END
}

slm_status slm_assign(slm_graph *g, int32_t *a_dev)
{
    API_BEGIN
    REQUIRE(g != nullptr && (a_dev != nullptr || g->n == 0), SLM_E_INVALID, "null argument");
    if (g->n == 0) return SLM_OK;
    LevelView L = view(g);
    run_assign(L, g->bins, a_dev, g->W.hub_ckey, g->W.hub_cid, g->s);
    API_END
}

static void load_assignment(slm_graph *g, const i32 *a_dev)
{
    HIPCHK(hipMemsetAsync(g->W.changed, 0, sizeof(int), g->s));
    k_label_range<<<small_grid(g->n), 256, 0, g->s>>>(a_dev, g->n, g->n, g->W.changed);
    HIPCHK(hipMemcpyAsync(g->W.h_scal, g->W.changed, sizeof(int), hipMemcpyDeviceToHost, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    REQUIRE(*(int *)g->W.h_scal == 0, SLM_E_INVALID, "assignment out of range");
    HIPCHK(hipMemcpyAsync(g->W.a, a_dev, sizeof(i32) * g->n, hipMemcpyDeviceToDevice, g->s));
}

slm_status slm_components(slm_graph *g, const int32_t *a_dev, int32_t *lab_dev,
                          uint8_t *on_cycle_dev, int64_t *n_c)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    REQUIRE(g->n == 0 || (a_dev && lab_dev), SLM_E_INVALID, "null argument");
    if (g->n == 0) {
        if (n_c) *n_c = 0;
        return SLM_OK;
    }
    load_assignment(g, a_dev);
    i64 nc = components(g->W, g->W.a, g->n, true, g->s);
    HIPCHK(hipMemcpyAsync(lab_dev, g->W.lab, sizeof(i32) * g->n, hipMemcpyDeviceToDevice, g->s));
    if (on_cycle_dev)
        HIPCHK(hipMemcpyAsync(on_cycle_dev, g->W.cyc, g->n, hipMemcpyDeviceToDevice, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    if (n_c) *n_c = nc;
    API_END
}

slm_status slm_positive(slm_graph *g, int32_t *a_dev, int64_t *splits)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    REQUIRE(g->n == 0 || a_dev, SLM_E_INVALID, "null argument");
    if (g->n == 0) {
        if (splits) *splits = 0;
        return SLM_OK;
    }
    load_assignment(g, a_dev);
    components(g->W, g->W.a, g->n, false, g->s);
    i64 nc;
    LevelView L = view(g);
    i64 sp = positive(g->W, L, g->bins, &nc, g->s);
    HIPCHK(hipMemcpyAsync(a_dev, g->W.a, sizeof(i32) * g->n, hipMemcpyDeviceToDevice, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    if (splits) *splits = sp;
    API_END
}

slm_status slm_sweep(slm_graph *g, const int32_t *lab_dev, int64_t n_c, int32_t *best_c_dev,
                     int64_t *delta_dev, int32_t *w_own_dev)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    if (g->n == 0) return SLM_OK;
    REQUIRE(best_c_dev && delta_dev && w_own_dev, SLM_E_INVALID, "null output");
    check_labels(g, lab_dev, n_c);
    LevelView L = view(g);
    community_totals(g->W, L, lab_dev, n_c, g->s);
    if (g->timing) HIPCHK(hipEventRecord(g->ev0, g->s));
    run_sweep(L, g->bins, lab_dev, g->W.sigma, best_c_dev, delta_dev, w_own_dev, g->W.hub_part,
              g->W.hub_poff, g->W.hub_cwin, g->W.hub_tkey, g->W.hub_tid, g->s,
              g->W.fan.use(g->nnz));
    if (g->timing) {
        HIPCHK(hipEventRecord(g->ev1, g->s));
        HIPCHK(hipEventSynchronize(g->ev1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, g->ev0, g->ev1));
        g->sweep_ms += ms;
        g->sweeps++;
        g->entries += g->nnz;
        g->bytes += 8 * g->nnz + 32 * g->n + 4 * n_c;
    }
    API_END
}

slm_status slm_round(slm_graph *g, const slm_params *p, int32_t level, int32_t round,
                     int32_t *a_dev, int64_t *stats)
{
    API_BEGIN
    REQUIRE(g != nullptr && p != nullptr, SLM_E_INVALID, "null argument");
    REQUIRE(g->n == 0 || a_dev, SLM_E_INVALID, "null assignment");
    REQUIRE(p->accept_p <= (1ull << 32), SLM_E_INVALID, "accept_p must be at most 2^32");
    if (g->n == 0) {
        if (stats) std::memset(stats, 0, sizeof(int64_t) * 4);
        return SLM_OK;
    }
    load_assignment(g, a_dev);
    batch_set_draws(g, p->seed, level);
    i64 nc = components(g->W, g->W.a, g->n, true, g->s);
    i64 st[4];
    level_round(g, p, level, round, &nc, st);
    HIPCHK(hipMemcpyAsync(a_dev, g->W.a, sizeof(i32) * g->n, hipMemcpyDeviceToDevice, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    if (stats) std::memcpy(stats, st, sizeof(st));
    API_END
}

slm_status slm_level(slm_graph *g, const slm_params *p, int32_t level, int32_t *lab_dev,
                     int64_t *n_c, int32_t *rounds, int32_t *converged)
{
    API_BEGIN
    REQUIRE(g != nullptr && p != nullptr, SLM_E_INVALID, "null argument");
    REQUIRE(g->n == 0 || lab_dev, SLM_E_INVALID, "null labels");
    REQUIRE(p->accept_p <= (1ull << 32), SLM_E_INVALID, "accept_p must be at most 2^32");
    if (g->n == 0) {
        if (n_c) *n_c = 0;
        if (rounds) *rounds = 0;
        if (converged) *converged = 1;
        return SLM_OK;
    }
    i64 nc;
    int32_t r, c;
    batch_set_draws(g, p->seed, level);
    run_level(g, p, level, &nc, &r, &c);
    HIPCHK(hipMemcpyAsync(lab_dev, g->W.lab, sizeof(i32) * g->n, hipMemcpyDeviceToDevice, g->s));
    HIPCHK(hipStreamSynchronize(g->s));
    if (n_c) *n_c = nc;
    if (rounds) *rounds = r;
    if (converged) *converged = c;
    API_END
}

slm_status slm_modularity(slm_graph *g, const int32_t *lab_dev, int64_t n_c, int64_t *nq,
                          double *q)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    REQUIRE(!g->is_union, SLM_E_STATE, "a batch reports modularity per graph through slm_batch_run");
    i64 v = 0;
    if (g->n > 0) {
        check_labels(g, lab_dev, n_c);
        v = modularity_num(g->W, view(g), g->bins, lab_dev, n_c, g->s);
    }
    if (nq) *nq = v;
    if (q) *q = g->m2 > 0 && g->keyA > 0 ? (double)v / (double)g->keyA / (double)g->m2 : 0.0;
    API_END
}

slm_status slm_contract(slm_graph *g, const int32_t *lab_dev, int64_t n_c)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    REQUIRE(!g->is_union, SLM_E_STATE, "a batch contracts inside slm_batch_run");
    check_labels(g, lab_dev, n_c);
    do_contract(g, lab_dev, n_c);
    API_END
}

slm_status slm_run(slm_graph *g, const slm_params *p, slm_result **out)
{
    API_BEGIN
    REQUIRE(g != nullptr && p != nullptr && out != nullptr, SLM_E_INVALID, "null argument");
    REQUIRE(p->accept_p <= (1ull << 32), SLM_E_INVALID, "accept_p must be at most 2^32");
    REQUIRE(p->max_rounds >= 0 && p->max_levels >= 0, SLM_E_INVALID, "negative cap");
    REQUIRE(!g->is_union, SLM_E_STATE, "a batch handle runs with slm_batch_run");
    *out = nullptr;
    do_reset(g);
    slm_result *r = new slm_result();
    r->n0 = g->n0;
    try {
        launch_iota_i32(g->composed, g->n0, g->s);
        int level = 0;
        while (g->m2 > 0 && g->n > 0) {
            i64 nc;
            int32_t rounds, conv;
            run_level(g, p, level, &nc, &rounds, &conv);
            if (nc == g->n) break;  // the level partition is the identity
            compose_labels(g->composed, g->W.lab, g->n0, g->s);
            i64 nq = modularity_num(g->W, view(g), g->bins, g->W.lab, nc, g->s);
            std::vector<i32> lab(g->n0);
            HIPCHK(hipMemcpyAsync(lab.data(), g->composed, sizeof(i32) * g->n0,
                                  hipMemcpyDeviceToHost, g->s));
            HIPCHK(hipStreamSynchronize(g->s));
            r->labels.push_back(std::move(lab));
            r->nc.push_back(nc);
            r->nq.push_back(nq);
            r->q.push_back((double)nq / (double)g->keyA / (double)g->m2);
            r->rounds.push_back(rounds);
            r->conv.push_back(conv);
            level++;
            if (p->max_levels > 0 && level >= p->max_levels) break;
            do_contract(g, g->W.lab, nc);
        }
    } catch (...) {
        delete r;
        throw;
    }
    *out = r;
    API_END
}

// Classical Louvain (the sequential comparison method): local moving in id
// order with exact sequential semantics, then canonical labels.
static void louvain_labels(slm_graph *g, const slm_params *p, i64 *nc, int32_t *passes,
                           int32_t *conv)
{
    int cv = 0;
    i64 mv = 0;
    *passes = louvain_level(g->W, view(g), p->max_rounds, &cv, &mv, g->s);
    *conv = cv;
    *nc = canonical_labels(g->W, g->n, g->s);
}

static void louvain_checks(slm_graph *g, const slm_params *p)
{
    REQUIRE(p->max_rounds >= 0 && p->max_levels >= 0, SLM_E_INVALID, "negative cap");
    REQUIRE(!g->is_union, SLM_E_STATE, "classical Louvain runs on a plain handle");
    REQUIRE(g->mkind == SLM_MODEL_CONFIG && g->mnum == 1 && g->mden == 1, SLM_E_STATE,
            "classical Louvain runs under the default null model");
}

slm_status slm_louvain_level(slm_graph *g, const slm_params *p, int32_t *lab_dev, int64_t *n_c,
                             int32_t *passes, int32_t *converged)
{
    API_BEGIN
    REQUIRE(g != nullptr && p != nullptr, SLM_E_INVALID, "null argument");
    REQUIRE(g->n == 0 || lab_dev, SLM_E_INVALID, "null labels");
    louvain_checks(g, p);
    i64 nc = 0;
    int32_t ps = 0, cv = 1;
    if (g->n > 0) {
        louvain_labels(g, p, &nc, &ps, &cv);
        HIPCHK(hipMemcpyAsync(lab_dev, g->W.lab, sizeof(i32) * g->n, hipMemcpyDeviceToDevice,
                              g->s));
        HIPCHK(hipStreamSynchronize(g->s));
    }
    if (n_c) *n_c = nc;
    if (passes) *passes = ps;
    if (converged) *converged = cv;
    API_END
}

slm_status slm_louvain_run(slm_graph *g, const slm_params *p, slm_result **out)
{
    API_BEGIN
    REQUIRE(g != nullptr && p != nullptr && out != nullptr, SLM_E_INVALID, "null argument");
    louvain_checks(g, p);
    *out = nullptr;
    do_reset(g);
    slm_result *r = new slm_result();
    r->n0 = g->n0;
    try {
        launch_iota_i32(g->composed, g->n0, g->s);
        int level = 0;
        while (g->m2 > 0 && g->n > 0) {
            i64 nc;
            int32_t passes, conv;
            louvain_labels(g, p, &nc, &passes, &conv);
            if (nc == g->n) break;  // no node moved: the identity
            compose_labels(g->composed, g->W.lab, g->n0, g->s);
            i64 nq = modularity_num(g->W, view(g), g->bins, g->W.lab, nc, g->s);
            std::vector<i32> lab(g->n0);
            HIPCHK(hipMemcpyAsync(lab.data(), g->composed, sizeof(i32) * g->n0,
                                  hipMemcpyDeviceToHost, g->s));
            HIPCHK(hipStreamSynchronize(g->s));
            r->labels.push_back(std::move(lab));
            r->nc.push_back(nc);
            r->nq.push_back(nq);
            r->q.push_back((double)nq / (double)g->keyA / (double)g->m2);
            r->rounds.push_back(passes);
            r->conv.push_back(conv);
            level++;
            if (p->max_levels > 0 && level >= p->max_levels) break;
            do_contract(g, g->W.lab, nc);
        }
    } catch (...) {
        delete r;
        throw;
    }
    *out = r;
    API_END
}

slm_status slm_result_num_levels(const slm_result *r, int32_t *levels)
{
    API_BEGIN
    REQUIRE(r != nullptr && levels != nullptr, SLM_E_INVALID, "null argument");
    *levels = (int32_t)r->nc.size();
    API_END
}

slm_status slm_result_level(const slm_result *r, int32_t level, int64_t *n_c,
                            const int32_t **labels, int64_t *nq, double *q, int32_t *rounds,
                            int32_t *converged)
{
    API_BEGIN
    REQUIRE(r != nullptr, SLM_E_INVALID, "null result");
    REQUIRE(level >= 0 && level < (int32_t)r->nc.size(), SLM_E_INVALID, "level out of range");
    if (n_c) *n_c = r->nc[level];
    if (labels) *labels = r->labels[level].data();
    if (nq) *nq = r->nq[level];
    if (q) *q = r->q[level];
    if (rounds) *rounds = r->rounds[level];
    if (converged) *converged = r->conv[level];
    API_END
}

slm_status slm_result_times(const slm_result *r, int64_t *submit_ns, int64_t *done_ns)
{
    API_BEGIN
    REQUIRE(r != nullptr, SLM_E_INVALID, "null result");
    if (submit_ns) *submit_ns = r->t_submit_ns;
    if (done_ns) *done_ns = r->t_done_ns;
    API_END
}

void slm_result_free(slm_result *r)
{
    delete r;
}

slm_status slm_timing_enable(slm_graph *g, int enable)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    g->timing = enable != 0;
    API_END
}

slm_status slm_set_option(slm_graph *g, const char *name, int64_t value)
{
    API_BEGIN
    REQUIRE(g != nullptr && name != nullptr, SLM_E_INVALID, "null argument");
    const std::string k(name);
    if (k == "hub_table_bits") {
        REQUIRE(value >= 4 && value <= 30 && (1 << value) <= HUB_TH, SLM_E_INVALID,
                "hub_table_bits must be in 4..11");
        g->bins.hub_tbits = (int)value;
    } else if (k == "hub_pass_pairs") {
        REQUIRE(value >= 1 && value <= ((int64_t)1 << 30), SLM_E_INVALID,
                "hub_pass_pairs must be in 1..2^30");
        g->bins.hub_cap = (int)value;
    } else if (k.rfind("grid_", 0) == 0) {
        int b = -1;
        for (int q = BIN_64; q <= BIN_4096; q++)
            if (k == "grid_" + std::to_string(kBinMaxDeg[q])) b = q;
        REQUIRE(b >= 0, SLM_E_INVALID, "grid_<d> needs d in 64..4096, a bin's largest degree");
        REQUIRE(value >= 0 && value <= 65535, SLM_E_INVALID, "grid_<d> must be in 0..65535");
        g->bins.grid_cap[b] = (i32)value;
    } else if (k == "union_shrink_min_nodes") {
        REQUIRE(g->is_union, SLM_E_INVALID, "union_shrink_min_nodes applies to batch handles");
        g->shrink_min = value;
    } else if (k == "fanout_min_entries") {
        REQUIRE(value >= 0, SLM_E_INVALID, "fanout_min_entries must be >= 0");
        g->W.fan.min_entries = value;
    } else {
        REQUIRE(false, SLM_E_INVALID, "unknown option");
    }
    API_END
}

slm_status slm_timing_read(slm_graph *g, double *sweep_ms, int64_t *sweeps, int64_t *entries,
                           int64_t *bytes)
{
    API_BEGIN
    REQUIRE(g != nullptr, SLM_E_INVALID, "null handle");
    HIPCHK(hipStreamSynchronize(g->s));
    if (sweep_ms) *sweep_ms = g->sweep_ms;
    if (sweeps) *sweeps = g->sweeps;
    if (entries) *entries = g->entries;
    if (bytes) *bytes = g->bytes;
    g->sweep_ms = 0;
    g->sweeps = g->entries = g->bytes = 0;
    API_END
}

slm_status slm_batch_create(int32_t count, const slm_graph_desc *graphs, int validate,
                            void *hip_stream, const slm_allocator *alloc, slm_graph **out)
{
    slm_graph *g = nullptr;
    try {
        REQUIRE(out != nullptr, SLM_E_INVALID, "null output handle");
        *out = nullptr;
        REQUIRE(count >= 1 && graphs != nullptr, SLM_E_INVALID, "a batch needs at least one graph");
        std::vector<i64> base0(count + 1, 0), ebase(count + 1, 0), m2g(count, 0);
        for (int i = 0; i < count; i++) {
            const slm_graph_desc &d = graphs[i];
            REQUIRE(d.n >= 0 && d.nnz >= 0, SLM_E_INVALID, "negative size");
            REQUIRE(d.row_ptr != nullptr, SLM_E_INVALID, "null row_ptr");
            REQUIRE(d.nnz == 0 || (d.col && d.w), SLM_E_INVALID, "null col or w");
            base0[i + 1] = base0[i] + d.n;
            ebase[i + 1] = ebase[i] + d.nnz;
        }
        const i64 N = base0[count], NNZ = ebase[count];
        REQUIRE(N < ((i64)1 << 31) - 1, SLM_E_OVERFLOW, "the batch must hold fewer than 2^31 - 1 nodes");
        REQUIRE(NNZ < ((i64)1 << 40), SLM_E_OVERFLOW, "too many entries");
        std::vector<i64> rp_h(N + 1);
        std::vector<int2> e_h(NNZ);
        for (int i = 0; i < count; i++) {
            const slm_graph_desc &d = graphs[i];
            std::vector<i64> rp(d.row_ptr, d.row_ptr + d.n + 1);
            i64 m2 = 0;
            if (validate) {
                validate_host(d.n, d.nnz, rp, d.col, d.w, &m2);
            } else {
                REQUIRE(rp[0] == 0 && rp[d.n] == d.nnz, SLM_E_INVALID,
                        "row_ptr must start at 0 and end at nnz");
                for (i64 j = 0; j < d.nnz; j++) m2 += d.w[j];
            }
            REQUIRE(m2 < ((i64)1 << 31), SLM_E_OVERFLOW, "total weight M2 must be below 2^31");
            m2g[i] = m2;
            for (i64 v = 0; v < d.n; v++) rp_h[base0[i] + v] = ebase[i] + rp[v];
            const i32 off = (i32)base0[i];
            for (i64 j = 0; j < d.nnz; j++)
                e_h[ebase[i] + j] = make_int2(d.col[j] + off, d.w[j]);
        }
        rp_h[N] = NNZ;
        g = new slm_graph();
        g->s = (hipStream_t)hip_stream;
        set_allocator(g, alloc);
        HIPCHK(hipGetDevice(&g->device));
        g->n0 = g->n = N;
        g->nnz0 = g->nnz = NNZ;
        g->mem0.resize(count);
        for (int i = 0; i < count; i++) {
            Member &m = g->mem0[i];
            m.ticket = (u64)i;
            m.n0 = graphs[i].n;
            m.nnz0 = graphs[i].nnz;
            m.m2 = m2g[i];
        }
        g->base0 = base0;
        g->mem = g->mem0;
        g->base = base0;
        g->G = count;
        alloc_union(g, count);
        init_from_host(g, rp_h.data(), e_h.data());
        union_upload(g);
        union_meta(g, 0, g->gidL[2], g->m2nL[2]);
        HIPCHK(hipStreamSynchronize(g->s));
        *out = g;
        return SLM_OK;
    } catch (const SlmError &e) {
        if (g) slm_destroy(g);
        return fail(e);
    } catch (const std::bad_alloc &) {
        if (g) slm_destroy(g);
        return fail(SlmError{SLM_E_NOMEM, "host allocation failed"});
    }
}

slm_status slm_batch_size(const slm_graph *g, int32_t *count)
{
    API_BEGIN
    REQUIRE(g != nullptr && count != nullptr, SLM_E_INVALID, "null argument");
    *count = (int32_t)g->mem0.size();
    API_END
}

slm_status slm_batch_run(slm_graph *g, const slm_params *p, const uint64_t *seeds,
                         slm_result **outs)
{
    API_BEGIN
    REQUIRE(g != nullptr && p != nullptr && outs != nullptr, SLM_E_INVALID, "null argument");
    REQUIRE(g->is_union && !g->mem0.empty(), SLM_E_STATE, "not a batch handle (use slm_run)");
    REQUIRE(p->accept_p <= (1ull << 32), SLM_E_INVALID, "accept_p must be at most 2^32");
    REQUIRE(p->max_rounds >= 0 && p->max_levels >= 0, SLM_E_INVALID, "negative cap");
    const int count = (int)g->mem0.size();
    for (int i = 0; i < count; i++) outs[i] = nullptr;
    std::vector<slm_result *> res(count, nullptr);
    try {
        for (int i = 0; i < count; i++) res[i] = new slm_result();
        batch_run(g, p, seeds, res);
    } catch (...) {
        for (slm_result *r : res) delete r;
        throw;
    }
    for (int i = 0; i < count; i++) outs[i] = res[i];
    API_END
}

slm_status slm_batch_solve(int32_t count, const slm_graph_desc *graphs, const slm_params *p,
                           const uint64_t *seeds, void *hip_stream, const slm_allocator *alloc,
                           slm_result **outs)
{
    if (!p || !outs) {
        g_err = "null argument";
        return SLM_E_INVALID;
    }
    slm_graph *g = nullptr;
    for (int i = 0; i < count; i++) outs[i] = nullptr;
    slm_status st = slm_batch_create(count, graphs, p->validate, hip_stream, alloc, &g);
    if (st != SLM_OK) return st;
    st = slm_batch_run(g, p, seeds, outs);
    slm_destroy(g);
    return st;
}

// ================================================================== serving
}  // extern "C"

// A lane: one union engine on its own stream, driven by its own thread.
struct Lane {
    slm_graph *eng = nullptr;
    hipStream_t stream = nullptr;
    std::thread th;
    std::deque<Member> *queue = nullptr;  // the queue of its class (small or large graphs)
    bool dead = false;                    // stopped after a failure
    i64 cap_nodes = 0, cap_entries = 0;
    int cap_members = 0;
};

struct slm_server {
    slm_server_cfg cfg;
    slm_allocator alloc{};
    bool has_alloc = false;
    int device = 0;
    std::vector<Lane *> lanes;
    std::deque<Member> q_small, q_large;  // requests not yet admitted
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::unordered_map<u64, slm_result *> done;
    std::unordered_map<u64, std::string> failed;
    std::unordered_set<u64> open;  // submitted and not yet delivered
    std::unordered_set<u64> cancel_req;  // cancelled while resident in a lane
    std::unordered_set<u64> cancelled;   // cancelled, not yet reported
    u64 next_ticket = 1;
    bool stop = false;
    i64 submitted = 0, completed = 0;
};

// An empty union engine with room for cap_n nodes, cap_e entries and cap_m
// members at level 0 (contraction never grows a level).
static i64 now_ns()
{
    return (i64)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

static slm_graph *make_engine(i64 cap_n, i64 cap_e, int cap_m, hipStream_t s,
                              const slm_allocator *alloc)
{
    slm_graph *g = new slm_graph();
    try {
        g->s = s;
        set_allocator(g, alloc);
        g->no_fanout = true;
        HIPCHK(hipGetDevice(&g->device));
        g->n0 = cap_n;
        g->nnz0 = cap_e;
        alloc_work(g);
        alloc_union(g, cap_m);
        HIPCHK(hipEventCreate(&g->ev0));
        HIPCHK(hipEventCreate(&g->ev1));
        g->n = g->nnz = 0;
        g->G = 0;
        g->base.assign(1, 0);
        g->cur = 0;
        g->level = 1;  // strengths of later levels never reset M2
    } catch (...) {
        slm_destroy(g);
        throw;
    }
    return g;
}

// A failed level leaves the lane's graphs undefined: fail all of them, the
// resident ones, those taken from the queue but not yet in the union (`add`)
// and those that finished the level but were not handed over yet (`done`).
// A step that failed while moving members between these lists leaves
// moved-from entries behind, which keep their ticket and result pointer, so
// a ticket can appear in two lists: each is failed and its result freed once.
static void lane_fail(slm_server *sv, Lane *L, std::vector<Member> &add, std::vector<Member> &done,
                      const std::string &msg)
{
    slm_graph *g = L->eng;
    std::lock_guard<std::mutex> lk(sv->mu);
    std::unordered_set<u64> seen;
    for (std::vector<Member> *list : {&g->mem, &add, &done})
        for (Member &m : *list) {
            if (!m.res || !seen.insert(m.ticket).second) continue;
            if (sv->cancel_req.erase(m.ticket)) sv->cancelled.insert(m.ticket);
            else sv->failed[m.ticket] = msg;
            delete m.res;
        }
    g->mem.clear();
    add.clear();
    done.clear();
    g->G = 0;
    L->dead = true;
    // with no live lane left for its class, the class queue fails too
    bool live = false;
    for (Lane *o : sv->lanes) live |= (!o->dead && o->queue == L->queue);
    if (!live) {
        for (Member &m : *L->queue) {
            sv->failed[m.ticket] = msg;
            delete m.res;
        }
        L->queue->clear();
    }
    sv->cv_done.notify_all();
}

// Lane loop: at every level boundary admit queued requests (in order, while
// they fit the lane's free capacity), run one level for every resident
// graph in the same launches, and hand finished graphs to their tickets.
static void lane_loop(slm_server *sv, Lane *L)
{
    (void)hipSetDevice(sv->device);
    slm_graph *g = L->eng;
    std::vector<Member> add, done;
    try {
        while (true) {
            add.clear();
            {
                std::unique_lock<std::mutex> lk(sv->mu);
                sv->cv_work.wait(lk, [&] { return sv->stop || !L->queue->empty() || g->G > 0; });
                if (sv->stop && g->G == 0) break;
                i64 n = g->n, e = g->nnz;
                int G = g->G;
                while (!sv->stop && !L->queue->empty()) {
                    const Member &m = L->queue->front();
                    if (G + 1 > L->cap_members || n + m.n0 > L->cap_nodes ||
                        e + m.nnz0 > L->cap_entries)
                        break;
                    n += m.n0;
                    e += m.nnz0;
                    G++;
                    add.push_back(std::move(L->queue->front()));
                    L->queue->pop_front();
                }
            }
            const size_t nadd = add.size();
            if (!add.empty()) union_append(g, add);
            if (g->G == 0) continue;
            if (g->n == 0) {  // only graphs without nodes: no level
                for (Member &m : g->mem) done.push_back(std::move(m));
                g->mem.clear();
                g->base.assign(1, 0);
                g->G = 0;
            } else {
                const i64 t0 = now_ns();
                const int G0 = g->G;
                const i64 n0 = g->n, e0 = g->nnz;
                setup_level(g);
                const i64 t1 = now_ns();
                const std::function<void(std::vector<Member> &)> mark =
                    [sv](std::vector<Member> &mem) {
                        std::lock_guard<std::mutex> lk(sv->mu);
                        if (sv->cancel_req.empty()) return;
                        for (Member &m : mem) m.cancel |= sv->cancel_req.count(m.ticket) > 0;
                    };
                union_level(g, &sv->cfg.params, done, &mark);
                if (getenv("SLM_TRACE"))
                    fprintf(stderr, "lane %p level: G %d n %lld nnz %lld admitted %zu setup %.2f ms level %.2f ms done %zu\n",
                            (void *)L, G0, (long long)n0, (long long)e0, nadd, (t1 - t0) / 1e6,
                            (now_ns() - t1) / 1e6, done.size());
            }
            if (!done.empty()) {
                std::lock_guard<std::mutex> lk(sv->mu);
                const i64 t = now_ns();
                for (Member &m : done) {
                    if (sv->cancel_req.erase(m.ticket)) {
                        delete m.res;
                        sv->cancelled.insert(m.ticket);
                        continue;
                    }
                    m.res->t_done_ns = t;
                    sv->done[m.ticket] = m.res;
                    sv->completed++;
                }
                done.clear();
                sv->cv_done.notify_all();
            }
        }
    } catch (const SlmError &e) {
        lane_fail(sv, L, add, done, e.msg);
    } catch (const std::exception &e) {
        lane_fail(sv, L, add, done, std::string("host failure: ") + e.what());
    }
}

extern "C" {

slm_status slm_server_create(const slm_server_cfg *cfg, const slm_allocator *alloc,
                             slm_server **out)
{
    slm_server *sv = nullptr;
    try {
        REQUIRE(cfg != nullptr && out != nullptr, SLM_E_INVALID, "null argument");
        *out = nullptr;
        REQUIRE(cfg->lanes >= 1 && cfg->lanes <= 16, SLM_E_INVALID, "lanes must be 1..16");
        REQUIRE(cfg->large_lanes >= 0 && cfg->large_lanes < cfg->lanes, SLM_E_INVALID,
                "large_lanes must leave at least one lane for small graphs");
        REQUIRE(cfg->node_capacity >= 0 && cfg->entry_capacity >= 0 && cfg->max_members >= 0,
                SLM_E_INVALID, "negative capacity");
        REQUIRE(cfg->queue_cap >= 0, SLM_E_INVALID, "negative queue_cap");
        REQUIRE(!alloc || (alloc->alloc && alloc->free), SLM_E_INVALID,
                "an allocator needs both alloc and free");
        REQUIRE(cfg->params.accept_p <= (1ull << 32), SLM_E_INVALID, "accept_p must be at most 2^32");
        REQUIRE(cfg->params.max_rounds >= 0 && cfg->params.max_levels >= 0, SLM_E_INVALID,
                "negative cap");
        sv = new slm_server();
        sv->cfg = *cfg;
        if (alloc) {
            sv->alloc = *alloc;
            sv->has_alloc = true;
        }
        if (sv->cfg.node_capacity == 0) sv->cfg.node_capacity = (i64)1 << 22;
        if (sv->cfg.entry_capacity == 0) sv->cfg.entry_capacity = (i64)1 << 26;
        if (sv->cfg.max_members == 0) sv->cfg.max_members = 4096;
        REQUIRE(sv->cfg.node_capacity < ((i64)1 << 31) - 1, SLM_E_OVERFLOW, "node capacity too large");
        HIPCHK(hipGetDevice(&sv->device));
        for (int l = 0; l < sv->cfg.lanes; l++) {
            Lane *L = new Lane();
            sv->lanes.push_back(L);
            HIPCHK(hipStreamCreate(&L->stream));
            L->cap_nodes = sv->cfg.node_capacity;
            L->cap_entries = sv->cfg.entry_capacity;
            L->cap_members = sv->cfg.max_members;
            L->eng = make_engine(L->cap_nodes, L->cap_entries, L->cap_members, L->stream,
                                 sv->has_alloc ? &sv->alloc : nullptr);
            L->queue = l < sv->cfg.lanes - sv->cfg.large_lanes ? &sv->q_small : &sv->q_large;
        }
        for (Lane *L : sv->lanes) L->th = std::thread(lane_loop, sv, L);
        *out = sv;
        return SLM_OK;
    } catch (const SlmError &e) {
        if (sv) slm_server_destroy(sv);
        return fail(e);
    } catch (const std::bad_alloc &) {
        if (sv) slm_server_destroy(sv);
        return fail(SlmError{SLM_E_NOMEM, "host allocation failed"});
    }
}

slm_status slm_server_submit(slm_server *sv, const slm_graph_desc *d, uint64_t seed,
                             uint64_t *ticket)
{
    API_BEGIN
    REQUIRE(sv != nullptr && d != nullptr && ticket != nullptr, SLM_E_INVALID, "null argument");
    REQUIRE(d->n >= 0 && d->nnz >= 0 && d->row_ptr != nullptr, SLM_E_INVALID, "bad graph");
    REQUIRE(d->nnz == 0 || (d->col && d->w), SLM_E_INVALID, "null col or w");
    const bool large = sv->cfg.large_lanes > 0 && d->n > sv->cfg.large_nodes;
    REQUIRE(d->n <= sv->cfg.node_capacity && d->nnz <= sv->cfg.entry_capacity, SLM_E_NOMEM,
            "the graph exceeds the capacity of a lane");
    Member m;
    m.n0 = d->n;
    m.nnz0 = d->nnz;
    m.rp.assign(d->row_ptr, d->row_ptr + d->n + 1);
    if (sv->cfg.validate) {
        validate_host(d->n, d->nnz, m.rp, d->col, d->w, &m.m2);
    } else {
        REQUIRE(m.rp[0] == 0 && m.rp[d->n] == d->nnz, SLM_E_INVALID,
                "row_ptr must start at 0 and end at nnz");
        for (i64 j = 0; j < d->nnz; j++) m.m2 += d->w[j];
    }
    REQUIRE(m.m2 < ((i64)1 << 31), SLM_E_OVERFLOW, "total weight M2 must be below 2^31");
    m.col.assign(d->col, d->col + d->nnz);
    m.w.assign(d->w, d->w + d->nnz);
    m.seed = seed;
    m.comp.resize(d->n);
    for (i64 v = 0; v < d->n; v++) m.comp[v] = (i32)v;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        REQUIRE(!sv->stop, SLM_E_STATE, "the server is stopping");
        std::deque<Member> &q = large ? sv->q_large : sv->q_small;
        bool live = false;
        for (Lane *L : sv->lanes) live |= (!L->dead && L->queue == &q);
        REQUIRE(live, SLM_E_DEVICE, "every lane serving this graph's class has failed");
        REQUIRE(sv->cfg.queue_cap == 0 || (i64)q.size() < (i64)sv->cfg.queue_cap, SLM_E_BUSY,
                "the queue of this graph's class is full");
        m.res = new slm_result();
        m.res->n0 = d->n;
        m.res->t_submit_ns = now_ns();
        m.ticket = sv->next_ticket++;
        *ticket = m.ticket;
        sv->open.insert(m.ticket);
        q.push_back(std::move(m));
        sv->submitted++;
    }
    sv->cv_work.notify_all();
    API_END
}

static slm_status take_result(slm_server *sv, uint64_t ticket, slm_result **out, bool wait)
{
    std::unique_lock<std::mutex> lk(sv->mu);
    while (true) {
        if (!sv->open.count(ticket)) {
            g_err = "unknown or already delivered ticket";
            return SLM_E_INVALID;
        }
        auto it = sv->done.find(ticket);
        if (it != sv->done.end()) {
            *out = it->second;
            sv->done.erase(it);
            sv->open.erase(ticket);
            return SLM_OK;
        }
        if (sv->cancelled.erase(ticket)) {
            g_err = "the request was cancelled";
            sv->open.erase(ticket);
            return SLM_E_CANCELLED;
        }
        auto f = sv->failed.find(ticket);
        if (f != sv->failed.end()) {
            g_err = f->second;
            sv->failed.erase(f);
            sv->open.erase(ticket);
            return SLM_E_DEVICE;
        }
        if (!wait) {
            *out = nullptr;
            return SLM_OK;
        }
        sv->cv_done.wait(lk);
    }
}

slm_status slm_server_cancel(slm_server *sv, uint64_t ticket)
{
    API_BEGIN
    REQUIRE(sv != nullptr, SLM_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    REQUIRE(sv->open.count(ticket) > 0, SLM_E_INVALID, "unknown or already delivered ticket");
    if (sv->cancelled.count(ticket) || sv->cancel_req.count(ticket)) return SLM_OK;
    auto d = sv->done.find(ticket);
    if (d != sv->done.end()) {
        delete d->second;
        sv->done.erase(d);
        sv->cancelled.insert(ticket);
        sv->cv_done.notify_all();
        return SLM_OK;
    }
    if (sv->failed.erase(ticket)) {
        sv->cancelled.insert(ticket);
        sv->cv_done.notify_all();
        return SLM_OK;
    }
    for (std::deque<Member> *q : {&sv->q_small, &sv->q_large})
        for (auto it = q->begin(); it != q->end(); ++it)
            if (it->ticket == ticket) {
                delete it->res;
                q->erase(it);
                sv->cancelled.insert(ticket);
                sv->cv_done.notify_all();
                return SLM_OK;
            }
    sv->cancel_req.insert(ticket);  // resident: leaves at the end of its level
    API_END
}

slm_status slm_server_poll(slm_server *sv, uint64_t ticket, slm_result **out)
{
    API_BEGIN
    REQUIRE(sv != nullptr && out != nullptr, SLM_E_INVALID, "null argument");
    return take_result(sv, ticket, out, false);
    API_END
}

slm_status slm_server_wait(slm_server *sv, uint64_t ticket, slm_result **out)
{
    API_BEGIN
    REQUIRE(sv != nullptr && out != nullptr, SLM_E_INVALID, "null argument");
    return take_result(sv, ticket, out, true);
    API_END
}

slm_status slm_server_stats(slm_server *sv, int64_t *submitted, int64_t *completed,
                            int64_t *reserved_bytes)
{
    API_BEGIN
    REQUIRE(sv != nullptr, SLM_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (submitted) *submitted = sv->submitted;
    if (completed) *completed = sv->completed;
    if (reserved_bytes) {
        i64 b = 0;
        for (Lane *L : sv->lanes) b += L->eng ? L->eng->dm.held : 0;
        *reserved_bytes = b;
    }
    API_END
}

void slm_server_destroy(slm_server *sv)
{
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (Lane *L : sv->lanes)
        if (L->th.joinable()) L->th.join();
    for (Member &m : sv->q_small) delete m.res;
    for (Member &m : sv->q_large) delete m.res;
    for (Lane *L : sv->lanes) {
        if (L->eng) slm_destroy(L->eng);
        if (L->stream) (void)hipStreamDestroy(L->stream);
        delete L;
    }
    for (auto &kv : sv->done) delete kv.second;
    delete sv;
}

}  // extern "C"
