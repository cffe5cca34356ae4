// Work space of a handle and the host-side steps built on the forest
// kernels (components, POSITIVE, MAXIMAL resolution) and on the contraction
// kernels.
#pragma once

#include "slm_impl.h"

struct Work {
    DevMem *dm = nullptr;  // the handle's device memory
    i64 n0 = 0, nnz0 = 0;
    int kmax = 0;  // number of jump tables held

    // per node (n0 entries)
    i32 *a = nullptr, *lab = nullptr, *comp = nullptr, *best_c = nullptr, *w_own = nullptr;
    i32 *wc = nullptr, *sigma = nullptr, *k = nullptr, *diag = nullptr;
    i32 *y = nullptr, *sigy = nullptr;  // directed model: y and its totals
    i64 *suby = nullptr;                // directed model: subtree sums of y
    i64 *delta = nullptr;
    // moved: a node that moved in the last MAXIMAL round, or its old parent;
    // pact: per community id, holds such a node (its membership changed)
    uint8_t *moved = nullptr, *pact = nullptr;
    uint8_t *cyc = nullptr, *act = nullptr, *hasc = nullptr, *exam = nullptr,
            *exam_next = nullptr, *accept = nullptr, *head = nullptr;
    i32 *claim = nullptr, *L = nullptr, *pos = nullptr, *cnode = nullptr, *mlist = nullptr;
    // POSITIVE work space
    i32 *fidx = nullptr, *flist = nullptr, *fcnt = nullptr, *flen = nullptr, *mem = nullptr;
    i32 *ptmp = nullptr, *pord = nullptr, *pchl = nullptr, *plvl = nullptr;
    i32 *part = nullptr, *win = nullptr, *psub = nullptr, *pcut = nullptr, *pdep = nullptr,
        *proot = nullptr, *chs = nullptr, *chc = nullptr;
    i64 *mem_off = nullptr, *pdp = nullptr, *woff_f = nullptr, *noff_f = nullptr;
    i64 *wsz = nullptr, *nsz = nullptr;
    int4 *pstk = nullptr;
    Fanout fan;            // side streams of the sweep
    i32 *A0 = nullptr, *A1 = nullptr, *M0 = nullptr, *M1 = nullptr;
    i32 *J = nullptr;  // kmax tables of n0
    i32 *D0 = nullptr, *D1 = nullptr;
    i64 *S0 = nullptr, *S1 = nullptr, *subk = nullptr, *cut = nullptr, *key = nullptr;
    i64 *bestkey = nullptr, *cbest_key = nullptr, *woff = nullptr, *noff = nullptr;
    u64 *bestpair = nullptr, *cbest_pair = nullptr;
    i32 *nca0 = nullptr, *nca1 = nullptr, *wbd = nullptr;
    i32 *ccnt = nullptr, *cfill = nullptr, *clist = nullptr;
    i64 *coff = nullptr;
    i32 *minm = nullptr;
    i64 *rank = nullptr;    // n0 + 1
    i64 *scan_tmp = nullptr;
    i64 *W = nullptr;       // cycle matrices (grown on demand)
    i64 W_cap = 0;

    i64 *counters = nullptr;  // device, 8 entries
    i32 *stepf = nullptr;     // device, 64 entries: per doubling step, "changed something"
    int *changed = nullptr;   // device flag
    i64 *h_scal = nullptr;    // pinned host, 16 entries

    // per entry (nnz0)
    i32 *src = nullptr;  // row of every CSR entry
    u64 *rk0 = nullptr, *rk1 = nullptr;
    i32 *rv0 = nullptr, *rv1 = nullptr;
    i32 *cnt = nullptr;   // n0
    i64 *roff = nullptr;  // n0 + 1
    i64 *hist = nullptr;  // radix histograms
    i64 hist_cap = 0;
    i64 *bscan = nullptr;  // degree-bin counts and their scan
    i64 bscan_cap = 0;
    uint8_t *head_e = nullptr; // nnz0 segment heads
    i64 *rank_e = nullptr;     // nnz0 + 1

    // hub work space of the sweep (pairs, partition offsets, chunk weights)
    // and of ASSIGN / re-pointing (per-chunk best)
    int2 *hub_part = nullptr;
    i64 hub_part_cap = 0;
    i64 *hub_poff = nullptr;
    i64 hub_poff_cap = 0;
    i32 *hub_cwin = nullptr;
    i64 hub_cwin_cap = 0;
    i64 *hub_ckey = nullptr;
    i32 *hub_cid = nullptr;
    i64 hub_chunk_cap = 0;
    i64 *hub_tkey = nullptr;   // per partition
    i32 *hub_tid = nullptr;
    i64 hub_tile_cap = 0;
};

// Arguments of the workgroup-per-community POSITIVE kernel.
struct PosArgs {
    LevelView G;
    i32 *a;              // assignment (updated)
    uint8_t *cyc;        // cycle flags (updated)
    const i32 *flist;    // community id of every flagged community
    const i64 *mem_off;  // members of flagged community f: mem[mem_off[f] .. mem_off[f+1])
    i32 *mem;
    i32 *tmp, *ord;      // per-community scratch (n entries)
    i32 *chl;            // children arena (2n entries)
    i64 *dpre;           // degree prefixes (n + nflag entries)
    i32 *lvl;            // level starts (n + nflag entries)
    int4 *stk;           // part stack (n entries)
    i32 *part, *win, *subk, *cut, *dep, *root, *chs, *chc, *cpos;  // per node
    const i32 *lcyc;     // cycle length of every flagged community
    const i64 *woff;     // cycle weight matrix offsets (L*L entries when L >= 2)
    i64 *W;
    const i64 *noff;     // cycle node list offsets
    i32 *cn;
    i64 *splits;
    int *err;            // 0, or the first tripped loop bound
};
void launch_positive_wg(const PosArgs &A, i64 nflag, hipStream_t s);
// S = W + W^T of the directed matrix in (rp, e) (n rows, nnz entries),
// written back in place (e must hold 2 nnz entries; the records need 2 nnz
// slots of the work space), and y = num-free k_out - k_in of W.  Returns
// nnz(S).
i64 symmetrize_level(Work &W, i64 *rp, int2 *e, i64 n, i64 nnz, i32 *y, hipStream_t s);
// POSITIVE under the directed model (node strengths x and y).
void launch_positive_dir(const PosArgs &A, i64 nflag, hipStream_t s);

struct Forest {
    int K = 0;            // highest jump table index in use
    i32 *depth = nullptr;
    i32 *root = nullptr;
};

// Reads n device int64 values into W.h_scal (synchronises the stream).
void read_scalars(Work &W, const i64 *dev, int n, hipStream_t s);

// COMPONENTS (Sec. 3.2) of the assignment a: W.comp = cycle minimum of every
// node's component, W.cyc = cycle flags; with want_lab also the canonical
// labels W.lab.  Returns n_c (only when want_lab, else -1).
i64 components(Work &W, const i32 *a, i64 n, bool want_lab, hipStream_t s);

// Canonical labels of the node-id community ids in W.comp; returns n_c.
i64 canonical_labels(Work &W, i64 n, hipStream_t s);
// Classical Louvain local moving of one level (k_louvain.hip): W.comp gets
// the community names; returns the passes that moved a node.
int louvain_level(Work &W, const LevelView &L, int max_passes, int *converged, i64 *moves,
                  hipStream_t s);

// POSITIVE (Sec. 3.3) on W.a (modified).  Expects W.comp / W.cyc from
// components(); leaves W.lab canonical.  Returns splits; *nc = n_c.
i64 positive(Work &W, const LevelView &Lv, const Bins &B, i64 *nc, hipStream_t s,
             const uint8_t *active = nullptr);
// After the components of a MAXIMAL round's assignment: W.pact[c] = 1 for the
// communities holding a node that W.moved marks (the others are unchanged
// since the last POSITIVE, so none of their nodes has a negative gain).
void mark_changed_communities(Work &W, i64 n, hipStream_t s);

// One MAXIMAL round (Sec. 3.4) on W.a with the canonical labels W.lab (n_c
// communities): sweep, tails, validity, draws, re-pointing.  Returns the
// number of valid moves (0: nothing changed); stats[0..2] = candidates,
// valid, accepted.
i64 maximal_moves(Work &W, const LevelView &Lv, const Bins &B, i64 nc, u64 seed, int level,
                  int round, u64 accept_p, i64 *stats, hipStream_t s, bool timing,
                  hipEvent_t ev0, hipEvent_t ev1, float *sweep_ms,
                  unsigned long long *gvalid = nullptr);

// Community totals S_C (canonical labels).
void community_totals(Work &W, const LevelView &Lv, const i32 *lab, i64 nc, hipStream_t s);

// Modularity numerator N_Q of the labelling lab (Sec. 2.4).
i64 modularity_num(Work &W, const LevelView &Lv, const Bins &B, const i32 *lab, i64 nc,
                   hipStream_t s);
// Per-graph modularity parts of a batch: accI[g] = sum of w(C,C) and
// accS[g] = sum of S_C^2 over the communities of graph g, where graph g owns
// the labels [gcb[g], gcb[g+1]).  accI and accS (G entries) are overwritten.
void modularity_graphs(Work &W, const LevelView &Lv, const Bins &B, const i32 *lab, i64 nc,
                       int G, const i64 *gcb, i64 *accI, i64 *accS, hipStream_t s);

// composed[v] = lab[composed[v]]
void compose_labels(i32 *composed, const i32 *lab, i64 n0, hipStream_t s);

// Row ids of every CSR entry.
void fill_src(const LevelView &Lv, const Bins &B, i32 *src, hipStream_t s);

// AGGREGATE (Sec. 3.5): contraction of the level into rp_out / e_out
// (n_c rows); returns the entry count.
i64 contract_level(Work &W, const LevelView &Lv, const Bins &B, const i32 *lab, i64 nc,
                   i64 *rp_out, int2 *e_out, hipStream_t s);

// Strengths and diagonal of the level; returns M2.
i64 level_strengths(Work &W, const i64 *rp, const int2 *e, const Bins &B, i64 n, i32 *k,
                    i32 *diag, hipStream_t s);
void run_strength_binned(const i64 *rp, const int2 *e, const Bins &Bn, i32 *k, i32 *diag,
                         hipStream_t s);

// ---------------------------------------------------------------- batches
void batch_first_labels(const i32 *lab, const i64 *gbase, int G, i64 *first, hipStream_t s);
void batch_relabel(const i32 *lab, const i32 *gid, const i32 *m2n, const i64 *shift,
                   const i32 *newpos, i64 n, i32 *lab2, i32 *gid2, i32 *m2n2, hipStream_t s);
void batch_meta(const i64 *gbase, int p0, int count, const i64 *m2p, i64 max_nodes, i32 *gid,
                i32 *m2n, hipStream_t s);

// A union shrunk to the graphs that still move during a level: one record per
// kept graph (its first node, entry and label in the shrunk union and in the
// union it comes from), then a closing record whose nb_s / eb_s / lb_s are
// the shrunk union's node, entry and label counts.
struct SubMember {
    i64 nb_s, eb_s, lb_s;
    i64 nb_u, eb_u, lb_u;
};
// Per graph of a union: its first node and first label there, and its first
// node in the union the level started with.
struct SaveMember {
    i64 nb_u, lb_u, nb_f;
};
// out[q] = rp[gbase[q]] for q = 0..G.
void batch_member_rows(const i64 *rp, const i64 *gbase, int G, i64 *out, hipStream_t s);
// The shrunk union's CSR (rp_s, e_s) and round state (a_s, lab_s, cyc_s) from
// the union's, for the G records of sm.
void batch_sub_gather(const SubMember *sm, int G, i64 n_s, i64 e_s, const i64 *rp_u,
                      const int2 *e_u, const i32 *a_u, const i32 *lab_u, const uint8_t *cyc_u,
                      i64 *rp_s, int2 *e_s_out, i32 *a_s, i32 *lab_s, uint8_t *cyc_s,
                      hipStream_t s);
// saved[node's id in the starting union] = its label minus its graph's first
// label, for the n nodes of a union (gid: per node, its graph's position).
void batch_sub_save(const i32 *gid, i64 n, const i32 *lab, const SaveMember *sv, i32 *saved,
                    hipStream_t s);
// lab[v] = saved[v] + lbase[gid[v]] over the starting union's n nodes.
void batch_sub_restore(const i32 *gid, i64 n, const i32 *saved, const i64 *lbase, i32 *lab,
                       hipStream_t s);
