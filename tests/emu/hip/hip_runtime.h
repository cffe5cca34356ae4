// Host emulation of the device features one workgroup-per-community kernel
// uses, for tests only: one std::thread per lane, __syncthreads as a
// workgroup barrier, wavefront shuffles through a per-wavefront exchange
// buffer, device atomics as host atomics.  A kernel whose barriers are not
// uniform (threads passing different numbers of barriers) leaves threads
// waiting here; a watchdog then reports each thread's barrier sequence.
#pragma once
#include <barrier>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

struct dim3 {
    unsigned x = 1, y = 1, z = 1;
};
struct int2 {
    int x, y;
};
struct int4 {
    int x, y, z, w;
};
static inline int2 make_int2(int a, int b) { return int2{a, b}; }
static inline int4 make_int4(int a, int b, int c, int d) { return int4{a, b, c, d}; }
typedef int hipError_t;
#define hipSuccess 0
typedef struct ihipStream_t *hipStream_t;
typedef struct ihipEvent_t *hipEvent_t;
static inline const char *hipGetErrorString(hipError_t) { return "host emulation"; }
static inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static  // one workgroup at a time
#define __restrict__ __restrict

extern thread_local dim3 threadIdx;
extern thread_local dim3 blockIdx;
extern dim3 blockDim, gridDim;

struct EmuWave {
    std::barrier<> *bar;
    uint64_t buf[64];
};
extern std::barrier<> *emu_block_bar;
extern EmuWave *emu_waves;
extern std::vector<int> emu_seq[1024];  // per thread: source lines of its barriers
extern volatile long emu_progress;
extern int emu_skew_us;  // > 0: lanes other than 0 wait this long after a barrier;
                         // < 0: every lane waits a random 0..-emu_skew_us
extern thread_local uint64_t emu_rng;

void emu_sleep_us(int us);

static inline void emu_sync(int line)
{
    emu_seq[threadIdx.x].push_back(line);
    emu_block_bar->arrive_and_wait();
    __atomic_fetch_add(&emu_progress, 1, __ATOMIC_RELAXED);
    if (emu_skew_us > 0 && threadIdx.x != 0) emu_sleep_us(emu_skew_us);
    if (emu_skew_us < 0) {
        emu_rng ^= emu_rng << 13;
        emu_rng ^= emu_rng >> 7;
        emu_rng ^= emu_rng << 17;
        emu_sleep_us((int)(emu_rng % (uint64_t)(1 - emu_skew_us)));
    }
}
#define __syncthreads() emu_sync(__LINE__)

template <class T>
static inline T emu_xchg(T v, int src)
{
    EmuWave &W = emu_waves[threadIdx.x / 64];
    const int lane = threadIdx.x & 63;
    uint64_t b = 0;
    std::memcpy(&b, &v, sizeof(T));
    W.buf[lane] = b;
    W.bar->arrive_and_wait();
    const uint64_t r = W.buf[src];
    W.bar->arrive_and_wait();
    T out;
    std::memcpy(&out, &r, sizeof(T));
    return out;
}
template <class T>
static inline T __shfl_xor(T v, int mask, int width = 64)
{
    const int lane = threadIdx.x & 63;
    return emu_xchg(v, (lane & ~(width - 1)) | ((lane ^ mask) & (width - 1)));
}
template <class T>
static inline T __shfl_up(T v, unsigned d, int width = 64)
{
    const int lane = threadIdx.x & 63;
    return emu_xchg(v, ((lane & (width - 1)) >= (int)d) ? lane - (int)d : lane);
}
template <class T>
static inline T __shfl_down(T v, unsigned d, int width = 64)
{
    const int lane = threadIdx.x & 63;
    return emu_xchg(v, ((lane & (width - 1)) + (int)d < width) ? lane + (int)d : lane);
}
static inline int __clzll(long long v) { return v == 0 ? 64 : __builtin_clzll((unsigned long long)v); }
template <class T> static inline T min(T a, T b) { return b < a ? b : a; }
template <class T> static inline T max(T a, T b) { return a < b ? b : a; }
static inline long long min(long long a, int b) { return b < a ? b : a; }
static inline long long min(int a, long long b) { return b < a ? b : a; }

#define EMU_ORD __ATOMIC_SEQ_CST
static inline int atomicAdd(int *p, int v) { return __atomic_fetch_add(p, v, EMU_ORD); }
static inline unsigned long long atomicAdd(unsigned long long *p, unsigned long long v)
{
    return __atomic_fetch_add(p, v, EMU_ORD);
}
static inline int atomicSub(int *p, int v) { return __atomic_fetch_sub(p, v, EMU_ORD); }
static inline int atomicOr(int *p, int v) { return __atomic_fetch_or(p, v, EMU_ORD); }
static inline int atomicExch(int *p, int v) { return __atomic_exchange_n(p, v, EMU_ORD); }
static inline int atomicCAS(int *p, int c, int v)
{
    __atomic_compare_exchange_n(p, &c, v, false, EMU_ORD, EMU_ORD);
    return c;
}
static inline unsigned long long atomicMin(unsigned long long *p, unsigned long long v)
{
    unsigned long long o = __atomic_load_n(p, EMU_ORD);
    while (v < o && !__atomic_compare_exchange_n(p, &o, v, false, EMU_ORD, EMU_ORD)) {
    }
    return o;
}
static inline unsigned long long atomicMax(unsigned long long *p, unsigned long long v)
{
    unsigned long long o = __atomic_load_n(p, EMU_ORD);
    while (v > o && !__atomic_compare_exchange_n(p, &o, v, false, EMU_ORD, EMU_ORD)) {
    }
    return o;
}
