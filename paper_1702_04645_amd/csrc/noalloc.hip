// Modularity of a labelling of a device-resident CSR with no allocation:
// the entry point slm_modularity_noalloc (include/slm.h).  It computes what
// slm_modularity computes for a handle (Sec. 2.4: N_Q = M2 * sum_C w(C,C) -
// sum_C S_C^2, Q = N_Q / M2 / M2), for callers that cannot allocate device
// memory and so cannot create a handle.  Its work space -- four int64
// accumulators, an error flag and the community totals -- lives in one
// file-scope device array per GPU instead of memory taken per call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "slm.h"
#include "slm_impl.h"

std::string &slm_error_slot();

// Work space of every call on a GPU.  Layout (bytes):
//   [0, 8)    sum over entries with both ends in one community of A_uv
//   [8, 16)   M2 = sum of all entries
//   [16, 24)  sum_C S_C^2
//   [24, 28)  error flags (bit 0: label out of range, bit 1: column out of
//             range, bit 2: row_ptr inconsistent, bit 3: weight < 1)
//   [256, 256 + 4 * SLM_NOALLOC_MAX_COMMUNITIES)  S_C, one uint32 per community
#define NA_HEAD 256
static __device__ __align__(256) unsigned char scratch[NA_HEAD + 4 * (size_t)SLM_NOALLOC_MAX_COMMUNITIES];

// The address of `scratch` on each device, looked up once per device with
// that device current.  The array's host-side name is not a device address.
#define NA_MAX_DEV 64
static std::mutex na_mu;
static void *na_ptr[NA_MAX_DEV];

static void *scratch_on_current_device()
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NA_MAX_DEV)
        throw SlmError{SLM_E_DEVICE, "device index out of the supported range"};
    std::lock_guard<std::mutex> lk(na_mu);
    if (!na_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw SlmError{SLM_E_DEVICE, "no device address for the work space"};
        na_ptr[dev] = p;
    }
    return na_ptr[dev];
}

struct NaHead {
    unsigned long long in_w;   // sum of A_uv with lab u == lab v
    unsigned long long m2;     // sum of A_uv
    unsigned long long sq;     // sum of S_C^2
    unsigned int flags;
};

// Clears the accumulators and the totals of the n_c communities (a fill
// kernel rather than a memset, so the call can sit in a captured graph).
__global__ void k_na_clear(NaHead *h, u32 *sig, i64 nc)
{
    const i64 t0 = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 == 0) {
        h->in_w = 0;
        h->m2 = 0;
        h->sq = 0;
        h->flags = 0;
    }
    for (i64 c = t0; c < nc; c += (i64)gridDim.x * blockDim.x) sig[c] = 0;
}

// One group of 16 lanes per row: the row's strength k_u (added to S of u's
// community) and its entries inside u's community.  Every index is checked
// before it is used; a bad one sets a flag and is skipped.
#define NA_G 16
__global__ __launch_bounds__(SLM_BS) void k_na_rows(const i64 *__restrict__ rp,
                                                   const i32 *__restrict__ col,
                                                   const i32 *__restrict__ w,
                                                   const i32 *__restrict__ lab, i64 n, i64 nnz,
                                                   i64 nc, NaHead *h, u32 *__restrict__ sig)
{
    __shared__ unsigned long long s_in, s_m2;
    if (threadIdx.x == 0) {
        s_in = 0;
        s_m2 = 0;
    }
    __syncthreads();
    const int gl = threadIdx.x % NA_G;
    const i64 groups = (i64)gridDim.x * (SLM_BS / NA_G);
    unsigned flags = 0;
    i64 in_acc = 0, m2_acc = 0;
    for (i64 u = (i64)blockIdx.x * (SLM_BS / NA_G) + threadIdx.x / NA_G; u < n; u += groups) {
        i64 b = rp[u], e = rp[u + 1];
        if (b < 0 || e < b || e > nnz) flags |= 4u;
        b = b < 0 ? 0 : (b > nnz ? nnz : b);
        e = e < b ? b : (e > nnz ? nnz : e);
        const i32 cu = lab[u];
        const bool lu_ok = cu >= 0 && cu < nc;
        if (!lu_ok) flags |= 1u;
        i64 k = 0, in = 0;
        for (i64 j = b + gl; j < e; j += NA_G) {
            const i32 v = col[j];
            const i32 wt = w[j];
            if (wt < 1) flags |= 8u;
            k += wt;
            if (v < 0 || v >= n) {
                flags |= 2u;
                continue;
            }
            if (lab[v] == cu) in += wt;
        }
#pragma unroll
        for (int d = NA_G / 2; d > 0; d >>= 1) {
            k += __shfl_xor(k, d, NA_G);
            in += __shfl_xor(in, d, NA_G);
        }
        if (gl == 0) {
            m2_acc += k;
            in_acc += in;
            // S_C needs no more than 32 bits when M2 < 2^31 (checked on the
            // host afterwards); a wider sum only wraps in a call that fails
            if (lu_ok) atomicAdd(&sig[cu], (u32)k);
        }
    }
    if (gl == 0) {
        atomicAdd(&s_in, (unsigned long long)in_acc);
        atomicAdd(&s_m2, (unsigned long long)m2_acc);
    }
    if (flags) atomicOr(&h->flags, flags);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&h->in_w, s_in);
        atomicAdd(&h->m2, s_m2);
    }
}

// sum over communities of S_C^2.
__global__ __launch_bounds__(SLM_BS) void k_na_squares(const u32 *__restrict__ sig, i64 nc,
                                                      NaHead *h)
{
    unsigned long long acc = 0;
    for (i64 c = (i64)blockIdx.x * blockDim.x + threadIdx.x; c < nc;
         c += (i64)gridDim.x * blockDim.x)
        acc += (unsigned long long)sig[c] * (unsigned long long)sig[c];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(&h->sq, acc);
}

static unsigned na_grid(i64 items, int per_block)
{
    i64 g = (items + per_block - 1) / per_block;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (unsigned)g;
}

extern "C" slm_status slm_modularity_noalloc(int64_t n, int64_t nnz, const int64_t *row_ptr_dev,
                                             const int32_t *col_dev, const int32_t *w_dev,
                                             const int32_t *lab_dev, int64_t n_c, int64_t *nq,
                                             double *q, void *hip_stream)
{
    try {
        if (n < 0 || nnz < 0 || n_c < 0)
            throw SlmError{SLM_E_INVALID, "negative size"};
        if (n >= ((i64)1 << 31)) throw SlmError{SLM_E_OVERFLOW, "n must be below 2^31"};
        if (n_c > n) throw SlmError{SLM_E_INVALID, "community count out of range"};
        if (n_c > SLM_NOALLOC_MAX_COMMUNITIES)
            throw SlmError{SLM_E_INVALID,
                           "slm_modularity_noalloc takes at most " +
                               std::to_string((long long)SLM_NOALLOC_MAX_COMMUNITIES) +
                               " communities (its work space is fixed)"};
        if (n > 0 && (!row_ptr_dev || !lab_dev || (nnz > 0 && (!col_dev || !w_dev))))
            throw SlmError{SLM_E_INVALID, "null input array"};
        if (n == 0) {
            if (nq) *nq = 0;
            if (q) *q = 0.0;
            return SLM_OK;
        }
        hipStream_t s = (hipStream_t)hip_stream;
        unsigned char *base = (unsigned char *)scratch_on_current_device();
        NaHead *h = (NaHead *)base;
        u32 *sig = (u32 *)(base + NA_HEAD);
        k_na_clear<<<na_grid(n_c, SLM_BS), SLM_BS, 0, s>>>(h, sig, n_c);
        HIPCHK(hipGetLastError());
        k_na_rows<<<na_grid(n, SLM_BS / NA_G), SLM_BS, 0, s>>>(row_ptr_dev, col_dev, w_dev,
                                                               lab_dev, n, nnz, n_c, h, sig);
        HIPCHK(hipGetLastError());
        k_na_squares<<<na_grid(n_c, SLM_BS), SLM_BS, 0, s>>>(sig, n_c, h);
        HIPCHK(hipGetLastError());
        NaHead hh;
        HIPCHK(hipMemcpyAsync(&hh, h, sizeof(NaHead), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hh.flags & 4u) throw SlmError{SLM_E_INVALID, "row_ptr is not a CSR of nnz entries"};
        if (hh.flags & 2u) throw SlmError{SLM_E_INVALID, "column out of range"};
        if (hh.flags & 8u) throw SlmError{SLM_E_INVALID, "weight below 1"};
        if (hh.flags & 1u) throw SlmError{SLM_E_INVALID, "label out of range"};
        if (hh.m2 >= (1ull << 31)) throw SlmError{SLM_E_OVERFLOW, "M2 must be below 2^31"};
        const i64 m2 = (i64)hh.m2;
        const i64 v = m2 * (i64)hh.in_w - (i64)hh.sq;
        if (nq) *nq = v;
        if (q) *q = m2 > 0 ? (double)v / (double)m2 / (double)m2 : 0.0;
        return SLM_OK;
    } catch (const SlmError &e) {
        slm_error_slot() = e.msg;
        return (slm_status)e.status;
    }
}
