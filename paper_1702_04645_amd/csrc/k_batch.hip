// Batched execution: many independent graphs run as one disjoint union.
// Each graph keeps its own total weight, seed, level and local node numbers
// (carried by the per-node and per-graph arrays of LevelView), so its labels
// are those of a run on its own.  These kernels move the per-graph
// bookkeeping between levels: the first label of every graph, the removal of
// finished graphs before AGGREGATE (with the renumbering of the graphs that
// stay), the per-node graph data of graphs joining the union, and the
// shrinking of a union to the graphs that still move within a level.
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

// Record of sm whose range [F(q), F(q+1)) holds j, F = nb_s (FIELD 0) or
// eb_s (FIELD 1); F(0) = 0 <= j < F(G).  Records with empty ranges are never
// returned.
template <int FIELD>
__device__ __forceinline__ int sub_find(const SubMember *__restrict__ sm, int G, i64 j)
{
    int lo = 0, hi = G;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        const i64 f = FIELD == 0 ? sm[mid].nb_s : sm[mid].eb_s;
        if (f <= j) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ void k_member_rows(const i64 *__restrict__ rp, const i64 *__restrict__ gbase, int G,
                              i64 *__restrict__ out)
{
    FLAT_LOOP((i64)G + 1) out[j] = rp[gbase[j]];
}

// Node j of the shrunk union is node j - nb_s + nb_u of its graph's union;
// row offsets, pointers and labels move with the graph's bases.
__global__ void k_sub_nodes(const SubMember *__restrict__ sm, int G, i64 n_s,
                            const i64 *__restrict__ rp_u, const i32 *__restrict__ a_u,
                            const i32 *__restrict__ lab_u, const uint8_t *__restrict__ cyc_u,
                            i64 *__restrict__ rp_s, i32 *__restrict__ a_s,
                            i32 *__restrict__ lab_s, uint8_t *__restrict__ cyc_s)
{
    FLAT_LOOP(n_s)
    {
        const SubMember m = sm[sub_find<0>(sm, G, j)];
        const i64 v = j - m.nb_s + m.nb_u;
        rp_s[j] = rp_u[v] - m.eb_u + m.eb_s;
        a_s[j] = (i32)(a_u[v] - m.nb_u + m.nb_s);
        lab_s[j] = (i32)(lab_u[v] - m.lb_u + m.lb_s);
        cyc_s[j] = cyc_u[v];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) rp_s[n_s] = sm[G].eb_s;
}

// Entries keep their weight; a column moves with its graph's node base (an
// entry never leaves its graph).
__global__ void k_sub_entries(const SubMember *__restrict__ sm, int G, i64 e_s,
                              const int2 *__restrict__ e_u, int2 *__restrict__ e_out)
{
    FLAT_LOOP(e_s)
    {
        const SubMember m = sm[sub_find<1>(sm, G, j)];
        const int2 ed = e_u[j - m.eb_s + m.eb_u];
        e_out[j] = make_int2((i32)(ed.x - m.nb_u + m.nb_s), ed.y);
    }
}

__global__ void k_sub_save(const i32 *__restrict__ gid, i64 n, const i32 *__restrict__ lab,
                           const SaveMember *__restrict__ sv, i32 *__restrict__ saved)
{
    FLAT_LOOP(n)
    {
        const SaveMember m = sv[gid[j]];
        saved[j - m.nb_u + m.nb_f] = (i32)(lab[j] - m.lb_u);
    }
}

__global__ void k_sub_restore(const i32 *__restrict__ gid, i64 n, const i32 *__restrict__ saved,
                              const i64 *__restrict__ lbase, i32 *__restrict__ lab)
{
    FLAT_LOOP(n) lab[j] = (i32)(saved[j] + lbase[gid[j]]);
}

void batch_member_rows(const i64 *rp, const i64 *gbase, int G, i64 *out, hipStream_t s)
{
    k_member_rows<<<flat_grid((i64)G + 1), SLM_BS, 0, s>>>(rp, gbase, G, out);
}

void batch_sub_gather(const SubMember *sm, int G, i64 n_s, i64 e_s, const i64 *rp_u,
                      const int2 *e_u, const i32 *a_u, const i32 *lab_u, const uint8_t *cyc_u,
                      i64 *rp_s, int2 *e_s_out, i32 *a_s, i32 *lab_s, uint8_t *cyc_s,
                      hipStream_t s)
{
    if (G <= 0) return;
    k_sub_nodes<<<flat_grid(n_s), SLM_BS, 0, s>>>(sm, G, n_s, rp_u, a_u, lab_u, cyc_u, rp_s, a_s,
                                                  lab_s, cyc_s);
    if (e_s > 0) k_sub_entries<<<flat_grid(e_s), SLM_BS, 0, s>>>(sm, G, e_s, e_u, e_s_out);
}

void batch_sub_save(const i32 *gid, i64 n, const i32 *lab, const SaveMember *sv, i32 *saved,
                    hipStream_t s)
{
    if (n > 0) k_sub_save<<<flat_grid(n), SLM_BS, 0, s>>>(gid, n, lab, sv, saved);
}

void batch_sub_restore(const i32 *gid, i64 n, const i32 *saved, const i64 *lbase, i32 *lab,
                       hipStream_t s)
{
    if (n > 0) k_sub_restore<<<flat_grid(n), SLM_BS, 0, s>>>(gid, n, saved, lbase, lab);
}
