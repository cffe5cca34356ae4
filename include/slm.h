/*
 * slm.h -- C ABI of the MI355X (gfx950) implementation of the Synchronised
 * Louvain Method (Chiem, Havelange & Van Dooren, arXiv 1702.04645).
 *
 * The method (Algorithm 1 of the paper) works level by level on a weighted
 * graph G_t: ASSIGN (Sec. 3.1) points every node at its best neighbour,
 * COMPONENTS (Sec. 3.2) takes the weakly connected components of that
 * assignment graph as communities, POSITIVE (Sec. 3.3) splits communities
 * holding nodes of negative local gain by their best bisection, MAXIMAL
 * (Sec. 3.4) moves nodes -- with their tails -- to their best neighbouring
 * community, all at once, and AGGREGATE (Sec. 3.5) contracts communities
 * into the nodes of the next level.  The objective is the weighted
 * modularity Q_w of Sec. 2.4.
 *
 * Graph convention.  The input is an undirected graph given as a symmetric
 * CSR matrix A: positive int32 weights, columns strictly ascending in every
 * row, the diagonal A_ii stored once.  k_i = sum_j A_ij (diagonal included),
 * M2 = sum_i k_i (the m_w of Sec. 2.4 for a symmetric matrix).  M2 must be
 * below 2^31; every gain is then an exact int64 integer:
 *   pair(i,j) = M2*A_ij - k_i*k_j            join(i,C) = M2*w(i,C) - k_i*S_C
 *   stay(i)   = M2*w(i,c_i\i) - k_i*(S_ci - k_i)
 *   move(B: c->D) = M2*(w(B,D) - w(B,c\B)) - S_B*(S_D - S_c + S_B)
 *   split(P1,P2)  = S_P1*S_P2 - M2*w(P1,P2)
 * (S_X = sum of k over X, w(X,Y) = sum of A_uv over u in X, v in Y).  Ties
 * go to the lowest node id, the lowest community label, the lowest
 * (first, second) cut node.  Communities carry canonical labels: numbered
 * 0..n_c-1 in increasing order of their smallest member.
 *
 * Memory.  Pointers named *_dev are device pointers (HBM of the current HIP
 * device), owned by the caller; everything else is host memory.  The handle
 * owns its device copy of the graph and its work space, taken from the
 * caller's allocator (slm_allocator, e.g. a framework's caching allocator)
 * when one is given at creation, else from hipMalloc; slm_destroy returns it.
 *
 * Streams.  All device work of a handle runs on the stream given at
 * creation (NULL = the default stream).  Calls that return a device result
 * are stream-ordered; calls that return host values synchronise the stream.
 * A handle is used by one thread at a time; distinct handles are
 * independent.
 *
 * Errors.  Every call returns slm_status; slm_last_error() gives a message
 * for the calling thread's last failure.  SLM_E_INVALID leaves the handle
 * unchanged.
 */
#ifndef SLM_H
#define SLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SLM_OK = 0,
    SLM_E_INVALID = 1,  /* bad argument or CSR (asymmetric, unsorted, weight < 1, ...) */
    SLM_E_OVERFLOW = 2, /* M2 >= 2^31 or n >= 2^31                                     */
    SLM_E_NOMEM = 3,    /* device or host allocation failed                            */
    SLM_E_DEVICE = 4,   /* a HIP call failed                                           */
    SLM_E_STATE = 5,    /* call out of order (e.g. contracting to as many nodes)       */
    SLM_E_BUSY = 6,     /* a server queue is full: submit again later                  */
    SLM_E_CANCELLED = 7 /* the served request was cancelled                            */
} slm_status;

/* Device memory provider.  alloc(ctx, bytes, stream) returns device memory
 * of at least `bytes` bytes usable on `stream` (the handle's hipStream_t),
 * or NULL on failure (the call then fails with SLM_E_NOMEM and the handle,
 * if any, stays destroyable); free(ctx, p, stream) returns it.  A buffer is
 * freed only after the work queued on `stream` that uses it has finished.
 * The callbacks may run on any thread of the library (a server's lanes
 * call them from their own threads) and must be thread-safe.  ctx is passed
 * through unchanged.  The allocator must outlive every handle made with it. */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *p, void *stream);
} slm_allocator;

typedef struct slm_graph slm_graph;
typedef struct slm_result slm_result;

/* Parameters of a run.
 *   seed       stream of the acceptance draws (Sec. 3.4); a draw is the high
 *              half of SplitMix64 output number (level<<48 | round<<32 | node)+1
 *   accept_p   Q32 acceptance threshold: a valid move is accepted iff its
 *              draw < accept_p (2^31 = probability 1/2, 2^32 = always)
 *   max_rounds cap on MAXIMAL rounds per level (the loop of Algorithm 1 ends
 *              earlier when no move is valid)
 *   max_levels cap on emitted levels, 0 = no cap
 *   validate   1 = check the CSR (symmetry, sorted unique columns, weights)
 *              at slm_create */
typedef struct {
    uint64_t seed;
    uint64_t accept_p;
    int32_t max_rounds;
    int32_t max_levels;
    int32_t validate;
    int32_t reserved;
} slm_params;

/* Defaults: seed 0, accept_p 2^31, max_rounds 64, max_levels 0, validate 1. */
void slm_params_default(slm_params *p);

/* Creates a handle holding a device copy of the level-0 graph G(V, E) of
 * Algorithm 1 (weighted, Sec. 2.4).
 *   row_ptr        n+1 offsets, int32 (row_ptr_bytes = 4) or int64 (8)
 *   col, w         nnz columns and weights
 *   inputs_on_device  0: the three arrays are host memory; 1: device memory
 *   validate       1: check symmetry, sorted unique columns, weights >= 1
 *   hip_stream     hipStream_t for all device work (NULL = default stream)
 *   alloc          device memory provider (NULL = hipMalloc / hipFree)
 * The inputs are copied; the caller keeps ownership.  Errors: SLM_E_INVALID,
 * SLM_E_OVERFLOW (M2 or n too large), SLM_E_NOMEM (also when alloc returns
 * NULL; nothing is left allocated), SLM_E_DEVICE. */
slm_status slm_create(int64_t n, int64_t nnz, const void *row_ptr, int row_ptr_bytes,
                      const int32_t *col, const int32_t *w, int inputs_on_device,
                      int validate, void *hip_stream, const slm_allocator *alloc,
                      slm_graph **out);

/* Null model of the quality function (Sec. 2.2: the energy with alpha_ij
 * and beta_ij; Sec. 2.3: null models; Sec. 2.4: weighted modularity).
 *   SLM_MODEL_CONFIG  configuration model with resolution gamma = num/den:
 *                     the modularity above with the null-model term scaled
 *                     by gamma; gains are num * (den*M2*w - num*k*S).
 *                     num = den = 1 is the default model of slm_create.
 *   SLM_MODEL_ER      Erdos-Renyi null model p_ij = p = num/den (alpha = 1,
 *                     beta = p): gains are num * (den*w - num*n_P*n_R) for
 *                     node sets of n_P and n_R original nodes.
 *   SLM_MODEL_DIRECTED  the weighted modularity of Sec. 2.4 of a directed
 *                     graph W (out- and in-strengths) with resolution
 *                     gamma = num/den.  The input CSR is W itself (row i
 *                     holds the arcs leaving i; no symmetry asked); the
 *                     levels run on S = W + W^T, with x = num*(k_out+k_in)
 *                     and a second strength y = num*(k_out-k_in), since
 *                     k_out_i K_in_C + k_in_i K_out_C = (x_i X_C - y_i Y_C)/2.
 * Every gain keeps the form A*w(P,R) - (X_P*X_R - Y_P*Y_R) with strengths
 * x, y (y = 0 but for the directed model) summed over node sets and a scale
 * A (num*den*M2, or num*den for Erdos-Renyi; M2 = sum of S for the directed
 * model), so all tie rules and strict tests above are unchanged.
 * N_Q = A * sum_C w(C,C) - sum_C (X_C^2 - Y_C^2) and Q = N_Q / A / M2.
 * Bounds (SLM_E_OVERFLOW otherwise): sum of x at most 2^30 and A*M2 at most
 * 2^61 for any model other than the default. */
typedef enum { SLM_MODEL_CONFIG = 0, SLM_MODEL_ER = 1, SLM_MODEL_DIRECTED = 2 } slm_model_kind;
typedef struct {
    int32_t kind;
    int32_t reserved;
    int64_t num;
    int64_t den;
} slm_model;

/* slm_create under a null model (model NULL = the default).  The input is
 * the symmetric CSR of slm_create, or for SLM_MODEL_DIRECTED any CSR with
 * sorted unique columns and weights >= 1 (sum of W + W^T below 2^31); the
 * handle's level 0 is then S = W + W^T (slm_level_info, slm_export_level).
 * Batches and servers use the default model only.  Errors as slm_create, plus SLM_E_INVALID for an unknown kind
 * or num, den < 1. */
slm_status slm_create_model(int64_t n, int64_t nnz, const void *row_ptr, int row_ptr_bytes,
                            const int32_t *col, const int32_t *w, int inputs_on_device,
                            int validate, const slm_model *model, void *hip_stream,
                            const slm_allocator *alloc, slm_graph **out);

void slm_destroy(slm_graph *g);

/* Current level index, its node and entry counts, and M2 (the same at
 * every level, Sec. 3.5). */
slm_status slm_level_info(const slm_graph *g, int32_t *level, int64_t *n_t,
                          int64_t *nnz_t, int64_t *m2);

/* Drops every contracted level: the handle is back at level 0. */
slm_status slm_reset(slm_graph *g);

/* Copies the current level's CSR to host arrays (row_ptr int64[n_t+1],
 * col and w int32[nnz_t]); synchronises. */
slm_status slm_export_level(slm_graph *g, int64_t *row_ptr, int32_t *col, int32_t *w);

/* ASSIGN (Sec. 3.1): a_dev[i] = the neighbour j != i of largest pair(i,j)
 * (ties to the lowest j) when that pair is positive, else i.
 * a_dev: n_t entries. */
slm_status slm_assign(slm_graph *g, int32_t *a_dev);

/* COMPONENTS (Sec. 3.2): canonical labels of the weakly connected
 * components of {(i, a(i))}; optional cycle flags (1 = on the cycle of its
 * component).  Writes lab_dev (n_t), on_cycle_dev (n_t bytes, may be NULL)
 * and the community count (host; synchronises). */
slm_status slm_components(slm_graph *g, const int32_t *a_dev, int32_t *lab_dev,
                          uint8_t *on_cycle_dev, int64_t *n_c);

/* POSITIVE (Sec. 3.3): while a community holds a node of negative local
 * gain g(i) = stay(i), apply its best bisection of the assignment graph --
 * the self-assignment of one non-cycle node (its subtree splits off) or of
 * two cycle nodes (the cycle splits in two arcs) -- with the largest split
 * key, ties to the lowest (first, second) cut node.  Modifies a_dev in
 * place; *splits (host, may be NULL) = splits applied.  Synchronises. */
slm_status slm_positive(slm_graph *g, int32_t *a_dev, int64_t *splits);

/* MAXIMAL sweep (Sec. 3.4, first loop of the appendix MAXIMAL): for every
 * node at once, from the labelling lab_dev (canonical, n_c communities):
 *   best_c_dev[i] = argmax over neighbouring communities C != c_i of
 *                   join(i,C) (ties to the lowest C) if that beats stay(i),
 *                   else c_i
 *   delta_dev[i]  = join - stay for a move, else 0
 *   w_own_dev[i]  = w(i, c_i \ i)
 * No state of the handle changes.  Stream-ordered. */
slm_status slm_sweep(slm_graph *g, const int32_t *lab_dev, int64_t n_c, int32_t *best_c_dev,
                     int64_t *delta_dev, int32_t *w_own_dev);

/* One MAXIMAL round followed by POSITIVE (the body of the inner loop of
 * Algorithm 1) on the assignment a_dev (modified in place).  A node whose
 * best community differs is valid iff moving its tail -- the node and every
 * node with a path to it, the whole community for a cycle node -- has
 * move > 0; a valid node is accepted iff draw(seed, level, round, node) <
 * accept_p and then points at its best neighbour (largest pair, ties to the
 * lowest id) inside the target community.  All moves use the state before
 * the round.  stats (host, 4 entries, may be NULL): candidates, valid,
 * accepted, splits.  With no valid node nothing changes.  Synchronises. */
slm_status slm_round(slm_graph *g, const slm_params *p, int32_t level, int32_t round,
                     int32_t *a_dev, int64_t *stats);

/* One level: ASSIGN, COMPONENTS, POSITIVE, then rounds until none is valid
 * or max_rounds.  Writes the canonical labels (lab_dev, n_t entries) and
 * host values n_c, rounds, converged.  Synchronises. */
slm_status slm_level(slm_graph *g, const slm_params *p, int32_t level, int32_t *lab_dev,
                     int64_t *n_c, int32_t *rounds, int32_t *converged);

/* Modularity (Sec. 2.4) of a labelling of the current level:
 * N_Q = M2 * sum_C w(C,C) - sum_C S_C^2 (exact) and Q = N_Q / M2 / M2
 * (IEEE double, computed on the host).  Synchronises. */
slm_status slm_modularity(slm_graph *g, const int32_t *lab_dev, int64_t n_c, int64_t *nq,
                          double *q);

/* AGGREGATE (Sec. 3.5): replaces the current level by its contraction,
 * A'_CD = sum of A_uv over u in C, v in D (diagonal included), rows sorted
 * by column.  SLM_E_STATE when n_c == n_t.  Synchronises. */
slm_status slm_contract(slm_graph *g, const int32_t *lab_dev, int64_t n_c);

/* Full run of Algorithm 1 from level 0 (the handle is reset first): levels
 * until a level's partition is the identity (not emitted) or max_levels.
 * The result holds, per emitted level, the labels composed onto the
 * original nodes, n_c, N_Q, Q, rounds and the converged flag. */
slm_status slm_run(slm_graph *g, const slm_params *p, slm_result **out);

/* Classical Louvain, the sequential method the SLM builds on, which Sec. 6
 * names as the comparison the paper leaves open.  A level moves nodes one
 * at a time in id order, each to its best neighbouring community (largest
 * join, lowest name on ties; communities are named by the node they started
 * from during the level) when that beats stay, seeing every earlier move;
 * passes repeat until one moves nothing or p->max_rounds passes, then
 * AGGREGATE (Sec. 3.5) as in the SLM.  The result is exactly the sequential
 * one: chunks of nodes decide at once from the same state and only the
 * decisions no earlier move of their chunk could change are kept.
 * slm_louvain_level: one level on the current level of the handle; writes
 * canonical labels (lab_dev, n_t entries), n_c, the passes that moved a node
 * and the converged flag.  slm_louvain_run: the full run from level 0, with
 * the result of slm_run (rounds = passes per level).  Plain handles under
 * the default model only (SLM_E_STATE otherwise).  Synchronise. */
slm_status slm_louvain_level(slm_graph *g, const slm_params *p, int32_t *lab_dev, int64_t *n_c,
                             int32_t *passes, int32_t *converged);
slm_status slm_louvain_run(slm_graph *g, const slm_params *p, slm_result **out);

slm_status slm_result_num_levels(const slm_result *r, int32_t *levels);
/* labels: n_0 entries owned by the result. */
slm_status slm_result_level(const slm_result *r, int32_t level, int64_t *n_c,
                            const int32_t **labels, int64_t *nq, double *q,
                            int32_t *rounds, int32_t *converged);
/* For a served request: steady-clock times (ns) of its submission and of
 * the end of its last level; 0 for results of slm_run / slm_batch_run. */
slm_status slm_result_times(const slm_result *r, int64_t *submit_ns, int64_t *done_ns);
void slm_result_free(slm_result *r);

/* ---------------------------------------------------------------- batches
 * Many independent graphs in one handle: they are held as one disjoint union
 * and every kernel launch of a level serves all of them.  Each graph keeps
 * its own M2 (every key of its nodes uses it), its own seed, level and local
 * node numbers for the draws, and leaves the union when its level partition
 * is the identity or it has emitted max_levels levels; its result is
 * therefore the one slm_run gives for that graph alone with the same seed.
 * The batched run is an extension of the method for throughput; the paper
 * runs one graph at a time. */

/* A host-memory CSR (same convention as slm_create; row_ptr is int64). */
typedef struct {
    int64_t n, nnz;
    const int64_t *row_ptr;
    const int32_t *col;
    const int32_t *w;
} slm_graph_desc;

/* Creates a batch handle from count >= 1 host graphs (copied; the caller
 * keeps ownership).  Each graph's M2 must be below 2^31 and the batch must
 * hold fewer than 2^31 - 1 nodes.  validate, hip_stream and alloc as in
 * slm_create.  On a batch
 * handle slm_assign, slm_components, slm_positive, slm_sweep, slm_round and
 * slm_level act on the level-0 union (slm_round and slm_level draw with
 * the given seed and level for every graph); slm_run, slm_modularity and
 * slm_contract return SLM_E_STATE. */
slm_status slm_batch_create(int32_t count, const slm_graph_desc *graphs, int validate,
                            void *hip_stream, const slm_allocator *alloc, slm_graph **out);

/* Number of graphs of a batch handle (0 for a plain handle). */
slm_status slm_batch_size(const slm_graph *g, int32_t *count);

/* Full runs of Algorithm 1 for every graph of the batch.  seeds: one per
 * graph (host), or NULL for p->seed everywhere.  outs: host array of
 * count result pointers, each freed with slm_result_free.  Synchronises. */
slm_status slm_batch_run(slm_graph *g, const slm_params *p, const uint64_t *seeds,
                         slm_result **outs);

/* One call for a batch used once: slm_batch_create (p->validate decides the
 * CSR checks), slm_batch_run, slm_destroy.  Same arguments and results;
 * on failure no result is returned and nothing stays allocated. */
slm_status slm_batch_solve(int32_t count, const slm_graph_desc *graphs, const slm_params *p,
                           const uint64_t *seeds, void *hip_stream,
                           const slm_allocator *alloc, slm_result **outs);

/* ---------------------------------------------------------------- serving
 * A server runs requests as they arrive.  Each lane is a union engine (the
 * batched run above) with its own HIP stream and host thread; at every level
 * boundary it admits queued requests in order while they fit its free
 * capacity, runs one level for all resident graphs in the same launches, and
 * hands finished graphs to their tickets.  A graph keeps its CSR and labels
 * in HBM for its whole run.  Each result is the one slm_run gives for that
 * graph alone with the request's seed, whatever else is resident.  Lanes of
 * one class (small or large graphs) take requests from one shared queue, so
 * a lane held by a long level does not hold up arrivals while another lane
 * of its class reaches a level boundary; large graphs get lanes of their own
 * so their long levels overlap on the device with the small ones.  The
 * serving loop is an extension for throughput and latency; the paper runs
 * one graph at a time. */
typedef struct slm_server slm_server;

typedef struct {
    int64_t node_capacity;   /* nodes resident at once per lane (0: 2^22)       */
    int64_t entry_capacity;  /* CSR entries resident at once per lane (0: 2^26) */
    int32_t max_members;     /* graphs resident at once per lane (0: 4096)      */
    int32_t lanes;           /* lanes in all, 1..16                             */
    int64_t large_nodes;     /* graphs with more nodes are "large"              */
    int32_t large_lanes;     /* lanes kept for large graphs (0: one queue for all) */
    int32_t validate;        /* check every submitted CSR                       */
    int32_t queue_cap;       /* requests waiting per class at most (0: no cap)  */
    slm_params params;       /* accept_p, max_rounds, max_levels of every run   */
} slm_server_cfg;

/* Creates the lanes (each reserves HBM for its capacities at once; the sum is
 * reported by slm_server_stats) on the current device.  The streams are
 * created with the default priority.  alloc as in slm_create (every lane's
 * device memory comes from it; NULL = hipMalloc). */
slm_status slm_server_create(const slm_server_cfg *cfg, const slm_allocator *alloc,
                             slm_server **out);

/* Queues a host CSR (copied; the caller keeps ownership) with its draw seed.
 * SLM_E_NOMEM when it can never fit its lane; SLM_E_INVALID /
 * SLM_E_OVERFLOW as for slm_create; SLM_E_BUSY when queue_cap requests of
 * its class already wait (nothing is queued: submit again later);
 * SLM_E_DEVICE when every lane of its class has failed.  *ticket identifies
 * the result. */
slm_status slm_server_submit(slm_server *sv, const slm_graph_desc *g, uint64_t seed,
                             uint64_t *ticket);

/* Cancels a ticket that has not been delivered.  A queued request is dropped
 * at once; a resident one leaves its lane at the end of the level it is in
 * (the other graphs of the lane are not affected); a finished, undelivered
 * result is freed.  Poll or wait on the ticket then gives SLM_E_CANCELLED
 * once (and delivers the ticket).  SLM_E_INVALID for an unknown or delivered
 * ticket. */
slm_status slm_server_cancel(slm_server *sv, uint64_t ticket);

/* The result of a ticket (then owned by the caller, freed with
 * slm_result_free), or *out = NULL while it runs.  A ticket is delivered
 * once; an unknown or delivered ticket gives SLM_E_INVALID.  SLM_E_DEVICE
 * when its lane failed (message in slm_last_error); SLM_E_CANCELLED after
 * slm_server_cancel. */
slm_status slm_server_poll(slm_server *sv, uint64_t ticket, slm_result **out);

/* As slm_server_poll, but blocks until the result is there. */
slm_status slm_server_wait(slm_server *sv, uint64_t ticket, slm_result **out);

/* Requests submitted and completed so far, and the HBM bytes the lanes hold. */
slm_status slm_server_stats(slm_server *sv, int64_t *submitted, int64_t *completed,
                            int64_t *reserved_bytes);

/* Stops admitting, lets resident graphs finish, drops queued ones and frees
 * everything, undelivered results included. */
void slm_server_destroy(slm_server *sv);

/* Sweep timing: when enabled, every sweep records HIP events on the
 * handle's stream around its kernels.  slm_timing_read reports the summed
 * sweep time (ms), the number of sweeps, the CSR entries they read, and the
 * algorithmic bytes they moved (8 per entry, 32 per node, 4 per community),
 * then clears the counters.  Synchronises. */
slm_status slm_timing_enable(slm_graph *g, int enable);
slm_status slm_timing_read(slm_graph *g, double *sweep_ms, int64_t *sweeps,
                           int64_t *entries, int64_t *bytes);

/* Launch tuning of the MAXIMAL sweep (Sec. 3.4).  name:
 *   "hub_table_bits"      hub rows (more than 4096 entries) total their
 *                         distinct labels per partition of the label space
 *                         in an LDS table of 2^value slots, 4..11 (default 11);
 *   "hub_pass_pairs"      pairs one pass over such a partition takes, 1..2^30
 *                         (default 1536); a larger partition is cut into more
 *                         passes, and a pass that fills the table is cut again;
 *   "grid_<d>"            workgroups of the persistent kernel of the degree bin
 *                         whose largest degree is d (64, 128, ..., 4096),
 *                         0..65535 (0: the default);
 *   "fanout_min_entries"  the degree bins run on the handle's side streams at
 *                         levels of at least this many entries (default 2^22).
 *   "union_shrink_min_nodes"  batch handles only: a union of at least this many
 *                         nodes shrinks, within a level, to its graphs that
 *                         still move once the others (no valid move in their
 *                         last round: their state is final for the level) hold
 *                         half of its nodes (default 2^16; 0: any size; < 0:
 *                         never).
 * Results never depend on these.  Takes effect from the next sweep.
 * SLM_E_INVALID for an unknown name or a value out of range (nothing
 * changes). */
slm_status slm_set_option(slm_graph *g, const char *name, int64_t value);

/* Modularity of a labelling without a handle and without allocating: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc) and so cannot
 * create a handle.  Returns what slm_modularity returns for a handle at
 * level 0 of the same graph: N_Q = M2 * sum_C w(C,C) - sum_C S_C^2 (exact,
 * *nq) and Q = N_Q / M2 / M2 (IEEE double, *q), M2 = sum of all entries.
 *   n, nnz       nodes and entries of a symmetric CSR (the convention above)
 *   row_ptr_dev  int64[n+1] device offsets
 *   col_dev, w_dev  int32[nnz] device columns and weights (>= 1)
 *   lab_dev      int32[n] device labels, each in [0, n_c)
 *   n_c          community count, at most SLM_NOALLOC_MAX_COMMUNITIES
 *   hip_stream   stream of the call's kernels (NULL = default stream)
 * nq and q are host pointers (either may be NULL); the call synchronises
 * the stream.  It calls no allocator: its work space (the community totals
 * and a few accumulators) is one fixed array per GPU, held by the library
 * until the process ends.  Every call on a GPU uses that GPU's array, so
 * calls that overlap on one GPU (several threads or streams) race; calls in
 * sequence are independent (each clears what it uses).  The matrix is not
 * checked for symmetry; out-of-range labels or columns, an inconsistent
 * row_ptr or a weight below 1 give SLM_E_INVALID (detected inside the
 * kernels, which skip the bad index), M2 >= 2^31 gives SLM_E_OVERFLOW. */
#define SLM_NOALLOC_MAX_COMMUNITIES (1 << 22)
slm_status slm_modularity_noalloc(int64_t n, int64_t nnz, const int64_t *row_ptr_dev,
                                  const int32_t *col_dev, const int32_t *w_dev,
                                  const int32_t *lab_dev, int64_t n_c, int64_t *nq, double *q,
                                  void *hip_stream);

/* Message of the calling thread's last failed call. */
const char *slm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLM_H */
