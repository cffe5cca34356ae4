// Small device utilities: fills and a device-wide exclusive prefix sum.
#include "slm_impl.h"

template <typename T>
__global__ void k_fill(T *p, T v, i64 n)
{
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    i64 stride = (i64)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_scale_i32(i32 *p, i32 f, i64 n)
{
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    i64 stride = (i64)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] *= f;
}

__global__ void k_iota(i32 *p, i64 n)
{
    i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    i64 stride = (i64)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = (i32)i;
}

static unsigned fill_grid(i64 n)
{
    i64 g = (n + SLM_BS - 1) / SLM_BS;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

void launch_fill_i32(i32 *p, i32 v, i64 n, hipStream_t s)
{
    if (n > 0) k_fill<i32><<<fill_grid(n), SLM_BS, 0, s>>>(p, v, n);
}
void launch_scale_i32(i32 *p, i32 f, i64 n, hipStream_t s)
{
    if (n > 0) k_scale_i32<<<fill_grid(n), SLM_BS, 0, s>>>(p, f, n);
}
void launch_fill_i64(i64 *p, i64 v, i64 n, hipStream_t s)
{
    if (n > 0) k_fill<i64><<<fill_grid(n), SLM_BS, 0, s>>>(p, v, n);
}
void launch_fill_u8(uint8_t *p, uint8_t v, i64 n, hipStream_t s)
{
    if (n > 0) k_fill<uint8_t><<<fill_grid(n), SLM_BS, 0, s>>>(p, v, n);
}
void launch_iota_i32(i32 *p, i64 n, hipStream_t s)
{
    if (n > 0) k_iota<<<fill_grid(n), SLM_BS, 0, s>>>(p, n);
}

// ------------------------------------------------------------------ scan
// Tile = 256 threads x 8 consecutive items per thread.
#define SCAN_ITEMS 8
#define SCAN_TILE (SLM_BS * SCAN_ITEMS)

__device__ __forceinline__ i64 wave_incl_scan(i64 v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        i64 t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the block; returns the block total.
__device__ __forceinline__ i64 block_excl_scan(i64 v, i64 &total)
{
    __shared__ i64 wsum[SLM_BS / 64];
    i64 inc = wave_incl_scan(v);
    const int wid = threadIdx.x / 64, lane = threadIdx.x & 63;
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    i64 before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < SLM_BS / 64; w++) {
        if (w < wid) before += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

template <typename T>
__global__ void k_scan_reduce(const T *in, i64 n, i64 *bsum)
{
    i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_ITEMS;
    i64 s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++)
        if (base + j < n) s += (i64)in[base + j];
    i64 tot;
    block_excl_scan(s, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of nb block sums in place; bsum[nb] = total.
__global__ void k_scan_top(i64 *bsum, i64 nb)
{
    i64 carry = 0;
    for (i64 base = 0; base < nb; base += SLM_BS) {
        i64 i = base + threadIdx.x;
        i64 v = i < nb ? bsum[i] : 0;
        i64 tot;
        i64 ex = block_excl_scan(v, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

template <typename T>
__global__ void k_scan_apply(const T *in, i64 *out, i64 n, const i64 *bsum, i64 nb)
{
    i64 base = (i64)blockIdx.x * SCAN_TILE + (i64)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    i64 s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        v[j] = (base + j < n) ? in[base + j] : (T)0;
        s += (i64)v[j];
    }
    i64 tot;
    i64 ex = block_excl_scan(s, tot) + bsum[blockIdx.x];
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; j++) {
        if (base + j < n) out[base + j] = ex;
        ex += (i64)v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

i64 scan_tmp_elems(i64 n)
{
    return (n + SCAN_TILE - 1) / SCAN_TILE + 2;
}

template <typename T>
static void scan_impl(const T *in, i64 *out, i64 n, i64 *tmp, hipStream_t s)
{
    i64 nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb < 1) nb = 1;
    k_scan_reduce<T><<<(unsigned)nb, SLM_BS, 0, s>>>(in, n, tmp);
    k_scan_top<<<1, SLM_BS, 0, s>>>(tmp, nb);
    k_scan_apply<T><<<(unsigned)nb, SLM_BS, 0, s>>>(in, out, n, tmp, nb);
}

void launch_scan_i32(const i32 *in, i64 *out, i64 n, i64 *tmp, hipStream_t s)
{
    scan_impl<i32>(in, out, n, tmp, s);
}
void launch_scan_i64(const i64 *in, i64 *out, i64 n, i64 *tmp, hipStream_t s)
{
    scan_impl<i64>(in, out, n, tmp, s);
}
void launch_scan_u8(const uint8_t *in, i64 *out, i64 n, i64 *tmp, hipStream_t s)
{
    scan_impl<uint8_t>(in, out, n, tmp, s);
}
