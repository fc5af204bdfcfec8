// Shared device/host helpers for the dd library (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dd.h"

namespace dd {

// ---------------------------------------------------------------------------
// error handling (host)
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// A failed call also leaves HIP's last-error state set; it is cleared here,
// since the exception reports it (else the next launch_check of a later call
// would report this error again).
#define DD_HIP(x)                                                                      \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) {                                                        \
            (void)hipGetLastError();                                                   \
            int c_ = (e_ == hipErrorOutOfMemory) ? DD_ERR_OOM : DD_ERR_HIP;            \
            throw ::dd::Error(c_, std::string(#x) + ": " + hipGetErrorString(e_));     \
        }                                                                              \
    } while (0)

#define DD_CHECK(cond, code, msg)                  \
    do {                                           \
        if (!(cond)) throw ::dd::Error(code, msg); \
    } while (0)

inline void launch_check(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error(DD_ERR_HIP, std::string("launch ") + what + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// device memory owned by RAII buffers, through the library's device cache:
// a setup allocates and frees tens of GB in a few hundred blocks, and
// hipMalloc of a large block has been seen to stall for seconds once the
// device has gone through a few such cycles.  Freed blocks are therefore kept
// per device and size class and handed to later requests (dev_alloc, dev_free
// in dd.hip; dd_trim_device_cache returns them).
// ---------------------------------------------------------------------------
void* dev_alloc(size_t bytes);              // throws Error(DD_ERR_OOM / DD_ERR_HIP)
void dev_free(void* p, size_t bytes) noexcept;
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) p = static_cast<T*>(dev_alloc(count * sizeof(T)));
    }
    void release() {
        if (p) dev_free(p, n * sizeof(T));
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

template <class T>
inline void h2d(T* d, const T* h, size_t n, hipStream_t s) {
    if (n) DD_HIP(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
inline void d2h(T* h, const T* d, size_t n, hipStream_t s) {
    if (n) DD_HIP(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
}
template <class T>
inline DBuf<T> upload(const std::vector<T>& v, hipStream_t s) {
    DBuf<T> b(v.size());
    h2d(b.p, v.data(), v.size(), s);
    DD_HIP(hipStreamSynchronize(s));  // host vector may die after return
    return b;
}

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// device reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// value of v in lane `lane` (uniform across the wave)
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane_t(double v, int lane) { return readlane_d(v, lane); }
__device__ __forceinline__ float readlane_t(float v, int lane) { return readlane_f(v, lane); }
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
// Block-wide sum; `red` must hold blockDim.x/64 doubles; result broadcast.
__device__ __forceinline__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    return s;
}
__device__ __forceinline__ double block_max(double v, double* red) {
    v = wave_max(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
    return s;
}

// ---------------------------------------------------------------------------
// Batched launches over uneven items: every item b contributes tiles(b) work
// units; a fixed grid walks the flattened unit list.  The prefix over items
// is recomputed in LDS by each workgroup (items <= kMaxItems).
// ---------------------------------------------------------------------------
constexpr int kMaxItems = 1024;

template <class Op>
__device__ __forceinline__ int item_prefix(const Op& op, int nitems, int* pre, int base) {
    // pre[0..nitems] = exclusive prefix of op.tiles(b); contiguous chunk per thread
    __shared__ int part[256];
    const int T = blockDim.x, t = threadIdx.x;
    const int chunk = (nitems + T - 1) / T;
    const int b0 = min(nitems, t * chunk), b1 = min(nitems, b0 + chunk);
    int s = 0;
    for (int b = b0; b < b1; ++b) {
        const int v = op.tiles(base + b);
        pre[b + 1] = v;
        s += v;
    }
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < T; off <<= 1) {
        const int add = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += add;
        __syncthreads();
    }
    int run = (t > 0) ? part[t - 1] : 0;
    for (int b = b0; b < b1; ++b) {
        run += pre[b + 1];
        pre[b + 1] = run;
    }
    if (t == 0) pre[0] = 0;
    __syncthreads();
    return pre[nitems];
}

__device__ __forceinline__ int find_item(const int* pre, int nitems, int t) {
    int lo = 0, hi = nitems;  // find largest b with pre[b] <= t, pre[b+1] > t
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Ops whose neighbouring tiles share operand panels and cost the same can opt
// in to an XCD-aware order (XcdChunked<Op>::value = true).  Workgroups are
// dispatched round-robin over the 8 XCDs, each with its own L2; such ops have
// their tiles taken in chunks of kXcdChunk consecutive tiles, chunk c on XCD
// c % 8, so that the tiles of one chunk hit in the same L2.
constexpr int kXcds = 8;
constexpr int kXcdChunk = 64;
template <class Op>
struct XcdChunked {
    static constexpr bool value = false;
};
// Ops built on mfma_tile_128 set this to 2: their kernel is compiled for two
// waves per SIMD (256 VGPRs), which holds the 64 x 64 accumulator of a wave.
template <class Op>
struct TileWaves {
    static constexpr int value = 0;
};

// Mapping of the tiles of one launch onto its workgroups (every mapping runs
// each tile once, by one workgroup, with the same arithmetic: the results do
// not depend on it).  TM_STATIC: workgroup g takes tiles g, g + G, ...;
// TM_XCD: the XCD-chunked order above; TM_LPT: a persistent work queue, every
// workgroup takes the next tile from a device counter until none is left, the
// items ordered by decreasing tile count (longest processing time first), so
// that the large subdomains start first and the small ones fill the end.
// TM_XLPT: the LPT order cut into chunks of kXcdChunk consecutive tiles,
// chunk c served by the workgroups of XCD c % 8 from a counter of that XCD
// (the XCD-chunked locality with dynamic balancing inside each XCD).
enum TileMode { TM_STATIC = 0, TM_XCD = 1, TM_LPT = 2, TM_XLPT = 3 };

constexpr int kLptItems = 256;  // the queue mode sorts at most this many items (small LDS footprint)
template <class Op>
__device__ __forceinline__ void tiles_lpt(const Op& op, int nitems, int base, int* counter, int* pre, bool xcd) {
    __shared__ int cnt[kLptItems], perm[kLptItems];
    __shared__ int tnext;
    int P = 1;
    while (P < nitems) P <<= 1;
    for (int b = threadIdx.x; b < P; b += blockDim.x) {
        cnt[b] = b < nitems ? op.tiles(base + b) : -1;
        perm[b] = b;
    }
    __syncthreads();
    // bitonic sort of (count descending, item ascending)
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const int ci = cnt[i], cl = cnt[l], pi = perm[i], pl = perm[l];
                    const bool i_first = ci > cl || (ci == cl && pi < pl);  // i before l in the wanted order
                    const bool up = (i & k) == 0;
                    if (up != i_first) {
                        cnt[i] = cl; cnt[l] = ci;
                        perm[i] = pl; perm[l] = pi;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        int run = 0;
        pre[0] = 0;
        for (int q = 0; q < nitems; ++q) {
            run += cnt[q];
            pre[q + 1] = run;
        }
    }
    __syncthreads();
    const int total = pre[nitems];
    if (xcd) {
        // counter[x] for the workgroups of XCD x (dispatch is round-robin over the
        // XCDs); every tile still runs once whatever the placement
        const int x = blockIdx.x % kXcds;
        for (;;) {
            if (threadIdx.x == 0) tnext = atomicAdd(counter + x, 1);
            __syncthreads();
            const int k = tnext;
            __syncthreads();
            const int c0 = (x + kXcds * (k / kXcdChunk)) * kXcdChunk;
            if (c0 >= total) break;  // later k of this XCD only visit later chunks
            const int t = c0 + k % kXcdChunk;
            if (t >= total) continue;
            const int q = find_item(pre, nitems, t);
            op(base + perm[q], t - pre[q]);
            __syncthreads();
        }
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) tnext = atomicAdd(counter, 1);
        __syncthreads();
        const int t = tnext;
        __syncthreads();
        if (t >= total) break;
        const int q = find_item(pre, nitems, t);
        op(base + perm[q], t - pre[q]);
        __syncthreads();
    }
}

template <class Op>
__device__ __forceinline__ void tiles_body(const Op& op, int nitems, int base, int mode, int* counter) {
    __shared__ int pre[kMaxItems + 1];
    if ((mode == TM_LPT || mode == TM_XLPT) && nitems <= kLptItems) {
        tiles_lpt(op, nitems, base, counter, pre, mode == TM_XLPT);
        return;
    }
    const int total = item_prefix(op, nitems, pre, base);
    const int G = gridDim.x, g = blockIdx.x;
    if (mode != TM_XCD || G % kXcds != 0 || G < kXcds * kXcdChunk) {
        for (int t = g; t < total; t += G) {
            const int b = find_item(pre, nitems, t);
            op(base + b, t - pre[b]);
            __syncthreads();
        }
        return;
    }
    const int x = g % kXcds, per = G / kXcds;
    for (int k = g / kXcds;; k += per) {
        const int c0 = (x + kXcds * (k / kXcdChunk)) * kXcdChunk;
        if (c0 >= total) break;  // later k only visit later chunks of this XCD
        const int t = c0 + k % kXcdChunk;
        if (t >= total) continue;
        const int b = find_item(pre, nitems, t);
        op(base + b, t - pre[b]);
        __syncthreads();
    }
}

template <class Op>
__global__ void __launch_bounds__(256) k_tiles(Op op, int nitems, int base, int mode, int* counter) {
    tiles_body(op, nitems, base, mode, counter);
}
// the same for ops that hold a 64 x 64 accumulator per wave (see TileWaves)
template <class Op>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_tiles_w2(Op op, int nitems, int base, int mode, int* counter) {
    tiles_body(op, nitems, base, mode, counter);
}
// Kernel meter: when armed with a launch name, every dispatch of that name is
// bracketed by a pair of HIP events on its own stream and its algorithmic
// work (flops, bytes) is recorded, so that the achieved rate of one kernel
// family can be read back without a profiler.  Process-wide, not thread-safe.
struct Meter {
    std::string name;
    std::vector<hipEvent_t> ev;     // start/stop pairs, in dispatch order
    std::vector<hipEvent_t> pool;   // recycled events
    double flops = 0.0, bytes = 0.0;
    int64_t launches = 0;
    bool armed(const char* n) const { return !name.empty() && name == n; }
    hipEvent_t get();
    void record_pair(hipEvent_t a, hipEvent_t b) { ev.push_back(a); ev.push_back(b); }
};
Meter& meter();

struct NoWork {
    void operator()(int, int, double&, double&) const {}
};

// Launch-mapping autotuner (dd.hip): for every launch name it tries the
// candidate mappings (TM_STATIC or TM_LPT at two grid caps, TM_XCD where the op
// allows it) on the launches as they come, times them with events, and keeps
// the fastest per tile once every candidate is measured (three samples, or one
// for a long launch or a launch name whose candidates are all cheap).  Disabled with
// DD_AUTOTUNE=0 (then TM_STATIC, or TM_XCD where the op opts in) and while a
// stream is being captured into a graph (then the decision so far is used).
struct TileChoice {
    int mode;
    int grid;
    int cand;  // candidate being sampled, -1 if none
};
TileChoice tile_choice(const char* name, bool xcd_ok, int max_grid, hipStream_t s);
void tile_sample(const char* name, int cand, hipEvent_t e0, hipEvent_t e1, int64_t tiles);
hipEvent_t tile_event();
int* tile_counter(int n = 1);  // n device counters of the current device (rotating slots), zeroed before use
__global__ void k_zero_counter(int* c, int n);

// Items are processed in chunks of kMaxItems (one launch per chunk).  work(base,
// cnt, flops, bytes) adds the algorithmic work of items [base, base+cnt); it is
// only called while the meter is armed for this launch name.
template <class Op, class Work = NoWork>
inline void launch_tiles(const Op& op, int nitems, int64_t total_hint, hipStream_t s, const char* name,
                         int max_grid = 4096, const Work& work = Work()) {
    if (nitems <= 0 || total_hint <= 0) return;
    const bool m = meter().armed(name);
    const TileChoice ch = tile_choice(name, XcdChunked<Op>::value, max_grid, s);
    for (int base = 0; base < nitems; base += kMaxItems) {
        const int cnt = std::min(kMaxItems, nitems - base);
        int grid = (int)std::min<int64_t>(total_hint, ch.grid);
        int* ctr = nullptr;
        int mode = ch.mode;
        if ((mode == TM_LPT || mode == TM_XLPT) && cnt > kLptItems) mode = TM_STATIC;
        if (mode == TM_XLPT && grid < kXcds) mode = TM_LPT;  // every XCD queue needs a workgroup
        if (mode == TM_LPT || mode == TM_XLPT) {
            const int nc = mode == TM_XLPT ? kXcds : 1;
            ctr = tile_counter(nc);
            hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, s, ctr, nc);
        }
        hipEvent_t e0 = nullptr, e1 = nullptr, t0 = nullptr, t1 = nullptr;
        if (m) {
            e0 = meter().get();
            e1 = meter().get();
            DD_HIP(hipEventRecord(e0, s));
        }
        if (ch.cand >= 0) {
            t0 = tile_event();
            t1 = tile_event();
            DD_HIP(hipEventRecord(t0, s));
        }
        if constexpr (TileWaves<Op>::value == 2)
            hipLaunchKernelGGL(k_tiles_w2<Op>, dim3(grid), dim3(256), 0, s, op, cnt, base, mode, ctr);
        else
            hipLaunchKernelGGL(k_tiles<Op>, dim3(grid), dim3(256), 0, s, op, cnt, base, mode, ctr);
        launch_check(name);
        if (ch.cand >= 0) {
            DD_HIP(hipEventRecord(t1, s));
            tile_sample(name, ch.cand, t0, t1, total_hint);
        }
        if (m) {
            DD_HIP(hipEventRecord(e1, s));
            meter().record_pair(e0, e1);
            work(base, cnt, meter().flops, meter().bytes);
            meter().launches++;
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 MFMA tile: 64x64 block tile, 4 waves of 32x32 (2x2 16x16x4 MFMA).
// Column-major operands.  op(A) is M x K, op(B) is K x N.
// Operand modes: 0 = plain; 1 = unit lower trapezoid stored below the
// diagonal (Householder vectors): stored (r,c) -> r<c ? 0 : r==c ? 1 : A(r,c).
// GATHER: op(A) row i is stored row ga[i] (no-transpose A only).
// ---------------------------------------------------------------------------
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double4_t mfma_f64(double a, double b, double4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// FP32 inputs and FP32 accumulation (the FP32 local factors)
typedef float float4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4_t mfma_f32(float a, float b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ double4_t mma16(double a, double b, double4_t c) { return mfma_f64(a, b, c); }
__device__ __forceinline__ float4_t mma16(float a, float b, float4_t c) { return mfma_f32(a, b, c); }
template <class T>
struct Vec4;
template <>
struct Vec4<double> {
    typedef double4_t type;
};
template <>
struct Vec4<float> {
    typedef float4_t type;
};
// Row of element e of lane l in the 16 x 16 result block (column l % 16 in
// both): the FP64 instruction interleaves the four elements over the lane
// groups, the FP32 one gives each lane group four consecutive rows.
__device__ __forceinline__ int acc_row(const double4_t*, int e, int l) { return 4 * e + (l >> 4); }
__device__ __forceinline__ int acc_row(const float4_t*, int e, int l) { return 4 * (l >> 4) + e; }

constexpr int KC = 16;  // K depth of one LDS stage

template <class T>
struct TileSmemT {
    T a[KC][64 + 1];
    T b[KC][64 + 1];
};
using TileSmem = TileSmemT<double>;

template <bool TA, int MODEA, class T>
__device__ __forceinline__ T load_a(const T* __restrict__ A, int64_t lda, int i, int k, int M, int K,
                                    const int* __restrict__ ga) {
    if (i >= M || k >= K) return T(0);
    int r = TA ? k : i, c = TA ? i : k;
    if (ga) r = ga[r];
    if (MODEA == 1) return (r < c) ? T(0) : (r == c ? T(1) : A[r + (int64_t)c * lda]);
    return A[r + (int64_t)c * lda];
}
template <bool TB, int MODEB, class T>
__device__ __forceinline__ T load_b(const T* __restrict__ B, int64_t ldb, int k, int j, int K, int N,
                                    const int* __restrict__ gb) {
    if (j >= N || k >= K) return T(0);
    int r = TB ? j : k, c = TB ? k : j;
    if (gb) r = gb[r];
    if (MODEB == 1) return (r < c) ? T(0) : (r == c ? T(1) : B[r + (int64_t)c * ldb]);
    return B[r + (int64_t)c * ldb];
}

// acc += op(A)[i0:i0+64, :] * op(B)[:, j0:j0+64].  K is consumed in stages of
// KC; the next stage's operands are loaded into registers while the MFMAs of
// the current stage run from LDS.
template <bool TA, bool TB, int MODEA = 0, int MODEB = 0, class T>
__device__ __forceinline__ void mfma_tile_64(const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                                             int64_t ldb, int M, int N, int K, int i0, int j0, TileSmemT<T>& sm,
                                             typename Vec4<T>::type (&acc)[2][2], const int* ga = nullptr,
                                             const int* gb = nullptr) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    constexpr int PER = (64 * KC) / 256;  // elements of each operand per thread and stage
    T ra[PER], rb[PER];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + q * 256;
            int ii, kk;
            if (!TA) { ii = e & 63; kk = e >> 6; } else { kk = e % KC; ii = e / KC; }
            ra[q] = load_a<TA, MODEA>(A, lda, i0 + ii, k0 + kk, M, K, ga);
            int jj, kb;
            if (!TB) { kb = e % KC; jj = e / KC; } else { jj = e & 63; kb = e >> 6; }
            rb[q] = load_b<TB, MODEB>(B, ldb, k0 + kb, j0 + jj, K, N, gb);
        }
    };
    if (K <= 0) return;
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + q * 256;
            int ii, kk;
            if (!TA) { ii = e & 63; kk = e >> 6; } else { kk = e % KC; ii = e / KC; }
            sm.a[kk][ii] = ra[q];
            int jj, kb;
            if (!TB) { kb = e % KC; jj = e / KC; } else { jj = e & 63; kb = e >> 6; }
            sm.b[kb][jj] = rb[q];
        }
        __syncthreads();
        if (k0 + KC < K) fetch(k0 + KC);
#pragma unroll 1
        for (int kq = 0; kq < KC / 4; ++kq) {
            const int kk = kq * 4 + (lane >> 4);
            const T a0 = sm.a[kk][wr + (lane & 15)], a1 = sm.a[kk][wr + 16 + (lane & 15)];
            const T b0 = sm.b[kk][wc + (lane & 15)], b1 = sm.b[kk][wc + 16 + (lane & 15)];
            acc[0][0] = mma16(a0, b0, acc[0][0]);
            acc[0][1] = mma16(a0, b1, acc[0][1]);
            acc[1][0] = mma16(a1, b0, acc[1][0]);
            acc[1][1] = mma16(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
}

template <class V>
__device__ __forceinline__ void acc_zero(V (&acc)[2][2]) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = V{0, 0, 0, 0};
}

// Stage the accumulator through LDS and hand it out in column-major order:
// f(row, col, value) is called with consecutive threads on consecutive rows
// of one column, so that the caller's global reads and writes of C are
// coalesced.  Reuses the tile's operand buffers (needs a sync before reuse).
// Operand buffers of the MFMA tile shared with a 64 x 65 staging area for
// the accumulator (epilogues that write C coalesced).
template <class T>
union TileSmemCT {
    TileSmemT<T> t;
    T c[64 * 65];
};
using TileSmemC = TileSmemCT<double>;

// acc -> LDS as a 64 x 64 column-major tile with ld 65; returns the buffer
// (synchronised: every thread may read any element).
template <class T>
__device__ __forceinline__ const T* acc_stage(const typename Vec4<T>::type (&acc)[2][2], TileSmemCT<T>& sm) {
    T* buf = sm.c;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
    __syncthreads();
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                buf[(wc + 16 * y + (lane & 15)) * 65 + wr + 16 * x + acc_row(&acc[0][0], j, lane)] = acc[x][y][j];
    __syncthreads();
    return buf;
}

template <class T, class F>
__device__ __forceinline__ void acc_store_coalesced(const typename Vec4<T>::type (&acc)[2][2], TileSmemCT<T>& sm,
                                                    F f) {
    const T* buf = acc_stage(acc, sm);
    const int r = threadIdx.x & 63;
#pragma unroll 4
    for (int c = threadIdx.x >> 6; c < 64; c += 4) f(r, c, buf[c * 65 + r]);
}

// Visit the accumulator: f(row, col, value) with tile-relative indices.  The
// element e of each lane is the entry at row acc_row(e, lane), column lane % 16.
template <class V, class F>
__device__ __forceinline__ void acc_foreach(const V (&acc)[2][2], F f) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int j = 0; j < 4; ++j) f(wr + 16 * x + acc_row(&acc[0][0], j, lane), wc + 16 * y + (lane & 15), acc[x][y][j]);
}


// ---------------------------------------------------------------------------
// FP64 MFMA tile, 128 x 128: 4 waves of 64 x 64 (4 x 4 MFMA 16x16x4 blocks),
// K consumed in stages of KC through two LDS buffers with one barrier per
// stage.  Same contract as mfma_tile_64 (column-major operands, transposes,
// operand mode 1 = unit lower trapezoid), without gathers.
//
// Full tiles with K a multiple of KC take a scheduled path: the whole stage is
// one basic block in which the next stage's global loads, the next k-step's
// LDS reads and the stage's LDS writes are interleaved with the MFMAs, so a
// wave's memory traffic overlaps its own matrix work (two waves per SIMD are
// too few to hide it otherwise).  Operands whose base is 16-byte aligned with
// an even leading dimension are read as double2.  Partial tiles take a
// bounds-checked path with the same accumulation order, so every element sees
// its K products summed in the same sequence whichever path computed it.
//
// The MFMA's first operand is taken from op(B) and its second from op(A), so
// that lane l of element e of acc[x][y] holds the tile entry (row 16y + l%16,
// column 16x + 4e + l/16) of its wave's 64 x 64 block: consecutive lanes hold
// consecutive rows of a column, and a column-major epilogue is coalesced.
// Ops that use it launch with two waves per SIMD (TileWaves).
// ---------------------------------------------------------------------------
struct TileSmem128 {
    double a[2][KC][128 + 1];
    double b[2][KC][128 + 1];
};
typedef double4_t Acc128[4][4];

template <class T>
__device__ __forceinline__ T gload(const T* p) {
    return *(const __attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ void acc128_zero(Acc128& acc) {
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = double4_t{0.0, 0.0, 0.0, 0.0};
}

// f(row, col, value), tile-relative; consecutive lanes visit consecutive rows
template <class F>
__device__ __forceinline__ void acc128_foreach(const Acc128& acc, F f) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w & 1) * 64, wc = (w >> 1) * 64;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) f(wr + 16 * y + (l & 15), wc + 16 * x + 4 * e + (l >> 4), acc[x][y][e]);
}

// stored (r, c) under operand mode 1: the unit lower trapezoid
template <int MODE>
__device__ __forceinline__ double mode_sel(double v, int r, int c) {
    if (MODE == 1) return (r < c) ? 0.0 : (r == c ? 1.0 : v);
    return v;
}

// One operand of the tile: rows `idx` (M or N index, 128) by KC.  CONTIG_IDX:
// the tile index is the contiguous storage direction (A not transposed, B
// transposed); otherwise K is.  Stored (r, c) = (idx, k) if CONTIG_IDX else
// (k, idx).  EDGE: entries with idx >= lim_i or k >= lim_k read a clamped
// (valid) address and are replaced by zero, without branches.
template <bool CONTIG_IDX, int MODE, bool VEC, bool EDGE>
struct TileOperand {
    const double* p;
    int64_t ld;
    int idx0, lim_i, lim_k;
    double2_t r[4];  // 128 x KC / 256 threads = 8 values, as 4 pairs
    __device__ __forceinline__ void map(int q, int& i, int& k) const {
        const int e = threadIdx.x + 256 * q;
        if (CONTIG_IDX) { i = (e & 63) * 2; k = e >> 6; }
        else { k = (e & (KC / 2 - 1)) * 2; i = e >> 3; }
    }
    __device__ __forceinline__ const double* at(int gi, int gk) const {
        return CONTIG_IDX ? p + gi + (int64_t)gk * ld : p + gk + (int64_t)gi * ld;
    }
    __device__ __forceinline__ void load(int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int i, k;
            map(q, i, k);
            const int gi = idx0 + i, gk = k0 + k;
            // the pair's second entry: next idx (CONTIG_IDX) or next k
            const int gi1 = CONTIG_IDX ? gi + 1 : gi, gk1 = CONTIG_IDX ? gk : gk + 1;
            if (EDGE) {
                const bool in0 = gi < lim_i && gk < lim_k, in1 = gi1 < lim_i && gk1 < lim_k;
                const double v0 = gload(at(min(gi, lim_i - 1), min(gk, lim_k - 1)));
                const double v1 = gload(at(min(gi1, lim_i - 1), min(gk1, lim_k - 1)));
                r[q][0] = in0 ? v0 : 0.0;
                r[q][1] = in1 ? v1 : 0.0;
            } else if (VEC) {
                r[q] = gload((const double2_t*)at(gi, gk));
            } else {
                r[q][0] = gload(at(gi, gk));
                r[q][1] = gload(at(gi, gk) + 1);  // the pair is contiguous in either layout
            }
            if (MODE == 1) {
                if (CONTIG_IDX) { r[q][0] = mode_sel<1>(r[q][0], gi, gk); r[q][1] = mode_sel<1>(r[q][1], gi1, gk1); }
                else { r[q][0] = mode_sel<1>(r[q][0], gk, gi); r[q][1] = mode_sel<1>(r[q][1], gk1, gi1); }
            }
        }
    }
    __device__ __forceinline__ void store(double (&s)[KC][128 + 1]) const {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int i, k;
            map(q, i, k);
            if (CONTIG_IDX) { s[k][i] = r[q][0]; s[k][i + 1] = r[q][1]; }
            else { s[k][i] = r[q][0]; s[k + 1][i] = r[q][1]; }
        }
    }
};

template <bool TA, bool TB, int MODEA, int MODEB, bool VA, bool VB, bool EDGE>
__device__ __forceinline__ void tile128_run(const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                                            int64_t ldb, int M, int N, int K, int i0, int j0, TileSmem128& sm,
                                            Acc128& acc) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wr = (w & 1) * 64, wc = (w >> 1) * 64;
    TileOperand<!TA, MODEA, VA, EDGE> oa{A, lda, i0, M, K};
    TileOperand<TB, MODEB, VB, EDGE> ob{B, ldb, j0, N, K};
    const int ns = (K + KC - 1) / KC;
    oa.load(0);
    ob.load(0);
    oa.store(sm.a[0]);
    ob.store(sm.b[0]);
    __syncthreads();
    for (int s = 0; s < ns; ++s) {
        const int buf = s & 1;
        const int kn = min(s + 1, ns - 1) * KC;  // the last stage reloads itself (unused)
        oa.load(kn);
        ob.load(kn);
        double fa[2][4], fb[2][4];
#pragma unroll
        for (int kq = 0; kq < KC / 4; ++kq) {
            if (kq == 0) {
                const int kk = l >> 4;
#pragma unroll
                for (int x = 0; x < 4; ++x) fb[0][x] = sm.b[buf][kk][wc + 16 * x + (l & 15)];
#pragma unroll
                for (int y = 0; y < 4; ++y) fa[0][y] = sm.a[buf][kk][wr + 16 * y + (l & 15)];
            }
            if (kq + 1 < KC / 4) {
                const int kk = (kq + 1) * 4 + (l >> 4), p = (kq + 1) & 1;
#pragma unroll
                for (int x = 0; x < 4; ++x) fb[p][x] = sm.b[buf][kk][wc + 16 * x + (l & 15)];
#pragma unroll
                for (int y = 0; y < 4; ++y) fa[p][y] = sm.a[buf][kk][wr + 16 * y + (l & 15)];
            }
            const int p = kq & 1;
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = mfma_f64(fb[p][x], fa[p][y], acc[x][y]);
        }
        oa.store(sm.a[buf ^ 1]);
        ob.store(sm.b[buf ^ 1]);
        // 64 MFMAs: a DS read after each of the first 24, the global loads
        // from the third on, the 16 DS writes with the last 16
#pragma unroll
        for (int i = 0; i < 64; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            if (i < 24) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            if (i >= 2 && i < (VA && VB ? 10 : 18)) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
            if (i >= 48) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
        }
        __syncthreads();
    }
}

// acc += op(A)[i0:i0+128, 0:K] * op(B)[0:K, j0:j0+128] (entries outside M x N
// are computed as zero rows/columns and must not be stored by the caller)
template <bool TA, bool TB, int MODEA = 0, int MODEB = 0>
__device__ __forceinline__ void mfma_tile_128(const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                                              int64_t ldb, int M, int N, int K, int i0, int j0, TileSmem128& sm,
                                              Acc128& acc) {
    if (K <= 0) return;
    if (i0 + 128 <= M && j0 + 128 <= N && K % KC == 0) {
        const bool va = (((uintptr_t)A & 15) == 0) && (lda & 1) == 0;
        const bool vb = (((uintptr_t)B & 15) == 0) && (ldb & 1) == 0;
        if (va && vb) tile128_run<TA, TB, MODEA, MODEB, true, true, false>(A, lda, B, ldb, M, N, K, i0, j0, sm, acc);
        else tile128_run<TA, TB, MODEA, MODEB, false, false, false>(A, lda, B, ldb, M, N, K, i0, j0, sm, acc);
    } else {
        tile128_run<TA, TB, MODEA, MODEB, false, false, true>(A, lda, B, ldb, M, N, K, i0, j0, sm, acc);
    }
}

// C[i0 + r, j0 + c] = alpha acc + beta C, for r < M - i0, c < N - j0 (loads
// of one x block issued before its stores)
__device__ __forceinline__ void acc128_axpby(const Acc128& acc, double* C, int64_t ld, int i0, int j0, int M, int N,
                                             double alpha, double beta) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r0 = i0 + (w & 1) * 64 + (l & 15), c0 = j0 + (w >> 1) * 64 + (l >> 4);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        double cv[4][4];
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = r0 + 16 * y, c = c0 + 16 * x + 4 * e;
                cv[y][e] = (r < M && c < N) ? gload(C + r + (int64_t)c * ld) : 0.0;
            }
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = r0 + 16 * y, c = c0 + 16 * x + 4 * e;
                if (r < M && c < N) C[r + (int64_t)c * ld] = alpha * acc[x][y][e] + beta * cv[y][e];
            }
    }
}

}  // namespace dd
