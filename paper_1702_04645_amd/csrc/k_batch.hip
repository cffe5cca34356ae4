// Batched execution: many independent graphs run as one disjoint union.
// Each graph keeps its own total weight, seed, level and local node numbers
// (carried by the per-node and per-graph arrays of LevelView), so its labels
// are those of a run on its own.  These kernels move the per-graph
// bookkeeping between levels: the first label of every graph, the masked
// composition of labels, the removal of finished graphs before AGGREGATE,
// and the per-node graph data of the next level.
#include "slm_forest.h"

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

// first[g] = lab[gbase[g]] for a graph with nodes at this level, else -1.
__global__ void k_first_label(const i32 *__restrict__ lab, const i64 *__restrict__ gbase, int G,
                              i64 *__restrict__ first)
{
    FLAT_LOOP(G) first[j] = gbase[j] < gbase[j + 1] ? (i64)lab[gbase[j]] : -1;
}

// composed[v] = lab[composed[v]] for the original nodes of graphs that emit
// this level (flag[gid0[v]] != 0).
__global__ void k_compose_masked(i32 *__restrict__ composed, const i32 *__restrict__ lab,
                                 const i32 *__restrict__ gid0, const uint8_t *__restrict__ flag,
                                 i64 n0)
{
    FLAT_LOOP(n0)
    {
        if (flag[gid0[j]]) composed[j] = lab[composed[j]];
    }
}

// Composed labels of the graphs that stay become node ids of the next level.
__global__ void k_compose_shift(i32 *__restrict__ composed, const i32 *__restrict__ gid0,
                                const i64 *__restrict__ shift, i64 n0)
{
    FLAT_LOOP(n0)
    {
        const i64 sh = shift[gid0[j]];
        if (sh > 0) composed[j] = (i32)(composed[j] - sh);
    }
}

// Labels for AGGREGATE: nodes of graphs that stay get lab - shift[g]
// (shift = communities of the graphs before g that leave); nodes of graphs
// that leave get -1.  The next level's per-node graph data is scattered to
// the community (every member writes the same value).
__global__ void k_batch_relabel(const i32 *__restrict__ lab, const i32 *__restrict__ gid,
                                const i32 *__restrict__ m2n, const i64 *__restrict__ shift, i64 n,
                                i32 *__restrict__ lab2, i32 *__restrict__ gid2,
                                i32 *__restrict__ m2n2)
{
    FLAT_LOOP(n)
    {
        const i32 g = gid[j];
        const i64 sh = shift[g];
        if (sh < 0) {
            lab2[j] = -1;
        } else {
            const i32 c = (i32)(lab[j] - sh);
            lab2[j] = c;
            gid2[c] = g;
            m2n2[c] = m2n[j];
        }
    }
}

// Per-node graph index and M2 of a freshly packed union.
__global__ void k_batch_meta(const i64 *__restrict__ gbase, int G, const i64 *__restrict__ m2g,
                             i32 *__restrict__ gid, i32 *__restrict__ m2n)
{
    const int g = blockIdx.y;
    if (g >= G) return;
    const i64 b = gbase[g], e = gbase[g + 1];
    for (i64 j = b + (i64)blockIdx.x * blockDim.x + threadIdx.x; j < e;
         j += (i64)gridDim.x * blockDim.x) {
        gid[j] = g;
        m2n[j] = (i32)m2g[g];
    }
}

void batch_first_labels(const i32 *lab, const i64 *gbase, int G, i64 *first, hipStream_t s)
{
    if (G > 0) k_first_label<<<flat_grid(G), SLM_BS, 0, s>>>(lab, gbase, G, first);
}

void batch_compose(i32 *composed, const i32 *lab, const i32 *gid0, const uint8_t *flag, i64 n0,
                   hipStream_t s)
{
    if (n0 > 0)
        k_compose_masked<<<flat_grid(n0), SLM_BS, 0, s>>>(composed, lab, gid0, flag, n0);
}

void batch_compose_shift(i32 *composed, const i32 *gid0, const i64 *shift, i64 n0,
                         hipStream_t s)
{
    if (n0 > 0) k_compose_shift<<<flat_grid(n0), SLM_BS, 0, s>>>(composed, gid0, shift, n0);
}

void batch_relabel(const i32 *lab, const i32 *gid, const i32 *m2n, const i64 *shift, i64 n,
                   i32 *lab2, i32 *gid2, i32 *m2n2, hipStream_t s)
{
    if (n > 0)
        k_batch_relabel<<<flat_grid(n), SLM_BS, 0, s>>>(lab, gid, m2n, shift, n, lab2, gid2,
                                                         m2n2);
}

void batch_meta(const i64 *gbase, int G, const i64 *m2g, i64 max_nodes, i32 *gid, i32 *m2n,
                hipStream_t s)
{
    if (G <= 0 || max_nodes <= 0) return;
    i64 gx = (max_nodes + SLM_BS - 1) / SLM_BS;
    if (gx > 64) gx = 64;
    dim3 grid((unsigned)gx, (unsigned)G);
    k_batch_meta<<<grid, SLM_BS, 0, s>>>(gbase, G, m2g, gid, m2n);
}
