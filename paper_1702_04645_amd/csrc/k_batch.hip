// Batched execution: many independent graphs run as one disjoint union.
// Each graph keeps its own total weight, seed, level and local node numbers
// (carried by the per-node and per-graph arrays of LevelView), so its labels
// are those of a run on its own.  These kernels move the per-graph
// bookkeeping between levels: the first label of every graph, the removal of
// finished graphs before AGGREGATE (with the renumbering of the graphs that
// stay), and the per-node graph data of graphs joining the union.
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

// Labels for AGGREGATE: nodes of graphs that stay get lab - shift[g]
// (shift = communities of the graphs before g that leave); nodes of graphs
// that leave get -1.  The next level's per-node graph data is scattered to
// the community (every member writes the same value); a graph that stays
// takes position newpos[g].
__global__ void k_batch_relabel(const i32 *__restrict__ lab, const i32 *__restrict__ gid,
                                const i32 *__restrict__ m2n, const i64 *__restrict__ shift,
                                const i32 *__restrict__ newpos, i64 n, i32 *__restrict__ lab2,
                                i32 *__restrict__ gid2, i32 *__restrict__ m2n2)
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
            gid2[c] = newpos[g];
            m2n2[c] = m2n[j];
        }
    }
}

// Per-node graph index and M2 for the graphs at positions p0 + blockIdx.y.
__global__ void k_batch_meta(const i64 *__restrict__ gbase, int p0, int count,
                             const i64 *__restrict__ m2p, i32 *__restrict__ gid,
                             i32 *__restrict__ m2n)
{
    if ((int)blockIdx.y >= count) return;
    const int g = p0 + (int)blockIdx.y;
    const i64 b = gbase[g], e = gbase[g + 1];
    const i32 m2 = (i32)m2p[g];
    for (i64 j = b + (i64)blockIdx.x * blockDim.x + threadIdx.x; j < e;
         j += (i64)gridDim.x * blockDim.x) {
        gid[j] = g;
        m2n[j] = m2;
    }
}

void batch_first_labels(const i32 *lab, const i64 *gbase, int G, i64 *first, hipStream_t s)
{
    if (G > 0) k_first_label<<<flat_grid(G), SLM_BS, 0, s>>>(lab, gbase, G, first);
}

void batch_relabel(const i32 *lab, const i32 *gid, const i32 *m2n, const i64 *shift,
                   const i32 *newpos, i64 n, i32 *lab2, i32 *gid2, i32 *m2n2, hipStream_t s)
{
    if (n > 0)
        k_batch_relabel<<<flat_grid(n), SLM_BS, 0, s>>>(lab, gid, m2n, shift, newpos, n, lab2,
                                                         gid2, m2n2);
}

void batch_meta(const i64 *gbase, int p0, int count, const i64 *m2p, i64 max_nodes, i32 *gid,
                i32 *m2n, hipStream_t s)
{
    if (count <= 0 || max_nodes <= 0) return;
    i64 gx = (max_nodes + SLM_BS - 1) / SLM_BS;
    if (gx > 64) gx = 64;
    for (int c0 = 0; c0 < count; c0 += 65535) {
        const int cnt = count - c0 < 65535 ? count - c0 : 65535;
        dim3 grid((unsigned)gx, (unsigned)cnt);
        k_batch_meta<<<grid, SLM_BS, 0, s>>>(gbase, p0 + c0, cnt, m2p, gid, m2n);
    }
}
