// Graph / index-map / extraction / vector kernels.
#include "sparse.hpp"

#include <algorithm>
#include <mutex>

namespace dd {

// ===========================================================================
// SplitMix64 (Steele, Lea & Flood 2014) and greedy graph growing
// ===========================================================================
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Seeds: sequential draw by a single thread (N is small compared with n).
__global__ void k_ggg_seeds(int64_t n, int N, uint64_t seed, int32_t* part, int32_t* round) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int chosen = 0;
    uint64_t k = 0;
    // every draw hits an untaken vertex with probability >= 1 - N/n, so the loop ends
    while (chosen < N) {
        const int64_t v = (int64_t)(splitmix64_at(seed, k++) % (uint64_t)n);
        if (part[v] < 0) {
            part[v] = chosen++;
            round[v] = 0;
        }
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Round r: unassigned v adjacent to a vertex assigned in round r-1 takes the
// minimum part id among those neighbours.
__global__ void k_ggg_round(CsrDev A, int32_t* part, int32_t* round, int r, int32_t* changed) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < A.n; v += (int64_t)gridDim.x * blockDim.x) {
        if (part[v] >= 0) continue;
        int best = 0x7fffffff;
        for (int e = A.rowptr[v]; e < A.rowptr[v + 1]; ++e) {
            const int c = A.colind[e];
            if (c != v && round[c] == r - 1) best = min(best, part[c]);
        }
        if (best != 0x7fffffff) {
            part[v] = best;
            round[v] = r;
            changed[0] = 1;
        }
    }
}

__global__ void k_part_sizes(const int32_t* part, int64_t n, int32_t* sizes) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (part[v] >= 0) atomicAdd(&sizes[part[v]], 1);
}

__global__ void k_ggg_rest(int32_t* part, int64_t n, const int32_t* sizes, int N) {
    __shared__ int target;
    if (threadIdx.x == 0) {
        int best = 0;
        for (int i = 1; i < N; ++i)
            if (sizes[i] < sizes[best]) best = i;
        target = best;
    }
    __syncthreads();
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        if (part[v] < 0) part[v] = target;
}

static int grid_for(int64_t n, int block = 256) { return (int)std::min<int64_t>((n + block - 1) / block, 65536); }

// The growing rule on caller-provided device buffers: round (n), sizes (N) and
// a flag (1).  Everything that must start at a value is set by fill kernels;
// the flag of every round comes back through *hflag (host memory).
static void ggg_run(const CsrDev& A, int N, uint64_t seed, int32_t* part, int32_t* round, int32_t* sizes,
                    int32_t* changed, int32_t* hflag, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(A.n)), dim3(256), 0, s, part, A.n, -1);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(A.n)), dim3(256), 0, s, round, A.n, -1);
    hipLaunchKernelGGL(k_ggg_seeds, dim3(1), dim3(1), 0, s, A.n, N, seed, part, round);
    launch_check("ggg_seeds");
    for (int r = 1;; ++r) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, changed, (int64_t)1, 0);
        hipLaunchKernelGGL(k_ggg_round, dim3(grid_for(A.n)), dim3(256), 0, s, A, part, round, r, changed);
        launch_check("ggg_round");
        DD_HIP(hipMemcpyAsync(hflag, changed, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        DD_HIP(hipStreamSynchronize(s));
        if (!*hflag) break;
    }
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(N)), dim3(256), 0, s, sizes, (int64_t)N, 0);
    hipLaunchKernelGGL(k_part_sizes, dim3(grid_for(A.n)), dim3(256), 0, s, part, A.n, sizes);
    hipLaunchKernelGGL(k_ggg_rest, dim3(grid_for(A.n)), dim3(256), 0, s, part, A.n, sizes, N);
    launch_check("ggg_rest");
    DD_HIP(hipStreamSynchronize(s));
}

void ggg_partition(const CsrDev& A, int N, uint64_t seed, int32_t* part, hipStream_t s) {
    DD_CHECK(N >= 1 && N <= A.n, DD_ERR_INVALID_ARG, "partition: need 1 <= N <= n");
    DBuf<int32_t> round(A.n), changed(1), sizes(N);
    int32_t* hchg = nullptr;
    DD_HIP(hipHostMalloc(&hchg, sizeof(int32_t)));
    try {
        ggg_run(A, N, seed, part, round.p, sizes.p, changed.p, hchg, s);
    } catch (...) {
        (void)hipHostFree(hchg);
        throw;
    }
    (void)hipHostFree(hchg);
}

// ---------------------------------------------------------------------------
// The same partition without any allocation, for callers that cannot allocate:
// its work arrays live in one file-scope device array per GPU.  In host code
// the array's name is not a device address; the address of each GPU's copy is
// taken once per device with hipGetSymbolAddress and only that is used.
// Calls that overlap on one GPU share the array and race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) int32_t scratch[kGggMaxN + kGggMaxParts + 64];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static int32_t* scratch_on_current_device() {
    int dev = 0;
    DD_HIP(hipGetDevice(&dev));
    DD_CHECK(dev >= 0 && dev < kMaxDevices, DD_ERR_INTERNAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        DD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        DD_CHECK(p != nullptr, DD_ERR_HIP, "no device address for the partition scratch array");
        g_scratch_ptr[dev] = static_cast<int32_t*>(p);
    }
    return g_scratch_ptr[dev];
}

void ggg_partition_noalloc(const CsrDev& A, int N, uint64_t seed, int32_t* part, hipStream_t s) {
    DD_CHECK(N >= 1 && N <= A.n, DD_ERR_INVALID_ARG, "partition: need 1 <= N <= n");
    DD_CHECK(A.n <= kGggMaxN, DD_ERR_INVALID_ARG, "partition without allocation: n beyond its scratch capacity");
    DD_CHECK(N <= kGggMaxParts, DD_ERR_INVALID_ARG, "partition without allocation: N beyond its scratch capacity");
    int32_t* base = scratch_on_current_device();
    int32_t* round = base;
    int32_t* sizes = base + kGggMaxN;
    int32_t* changed = base + kGggMaxN + kGggMaxParts;
    int32_t hflag = 0;
    ggg_run(A, N, seed, part, round, sizes, changed, &hflag, s);
}

__global__ void k_validate_part(const int32_t* part, int64_t n, int N, int32_t* counts, int32_t* bad) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int p = part[v];
        if (p < 0 || p >= N) atomicOr(bad, 1);
        else atomicAdd(&counts[p], 1);
    }
}

int validate_partition(const int32_t* part, int64_t n, int N, int32_t* dcounts, hipStream_t s) {
    DBuf<int32_t> bad(1);
    DD_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    DD_HIP(hipMemsetAsync(dcounts, 0, N * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_validate_part, dim3(grid_for(n)), dim3(256), 0, s, part, n, N, dcounts, bad.p);
    launch_check("validate_part");
    int32_t hb = 0;
    std::vector<int32_t> hc(N);
    DD_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DD_HIP(hipMemcpyAsync(hc.data(), dcounts, N * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    DD_HIP(hipStreamSynchronize(s));
    if (hb) return DD_ERR_INVALID_ARG;
    for (int i = 0; i < N; ++i)
        if (hc[i] == 0) return DD_ERR_INVALID_ARG;
    return DD_OK;
}

// ===========================================================================
// Overlap layers
// ===========================================================================
__global__ void k_dist_init(const int32_t* part, int64_t n, int N, uint8_t* dist) {
    const int64_t tot = n * (int64_t)N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n);
        const int64_t v = e % n;
        dist[e] = (part[v] == i) ? 0 : 255;
    }
}

// dist[i][v] = k for unvisited v with a neighbour at distance k-1 (writers agree)
__global__ void k_dist_layer(CsrDev A, int N, int k, uint8_t* dist) {
    const int64_t n = A.n, tot = n * (int64_t)N;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot; e += (int64_t)gridDim.x * blockDim.x) {
        if (dist[e] != 255) continue;
        const int i = (int)(e / n);
        const int64_t v = e % n;
        const uint8_t* di = dist + (int64_t)i * n;
        for (int q = A.rowptr[v]; q < A.rowptr[v + 1]; ++q) {
            const int c = A.colind[q];
            if (c != v && di[c] == k - 1) {
                dist[e] = (uint8_t)k;
                break;
            }
        }
    }
}

void layers(const CsrDev& A, const int32_t* part, int N, int delta, uint8_t* dist, hipStream_t s) {
    const int64_t tot = A.n * (int64_t)N;
    hipLaunchKernelGGL(k_dist_init, dim3(grid_for(tot)), dim3(256), 0, s, part, A.n, N, dist);
    for (int k = 1; k <= delta + 1; ++k)
        hipLaunchKernelGGL(k_dist_layer, dim3(grid_for(tot)), dim3(256), 0, s, A, N, k, dist);
    launch_check("layers");
}

__global__ void k_layer_counts(const uint8_t* dist, int64_t n, int delta, int32_t* counts) {
    const int i = blockIdx.x;
    const uint8_t* di = dist + (int64_t)i * n;
    int c0 = 0, c1 = 0, c2 = 0;
    for (int64_t v = threadIdx.x; v < n; v += blockDim.x) {
        const int d = di[v];
        c0 += (d == 0);
        c1 += (d >= 1 && d <= delta);
        c2 += (d == delta + 1);
    }
    __shared__ int s0, s1, s2;
    if (threadIdx.x == 0) { s0 = 0; s1 = 0; s2 = 0; }
    __syncthreads();
    atomicAdd(&s0, c0);
    atomicAdd(&s1, c1);
    atomicAdd(&s2, c2);
    __syncthreads();
    if (threadIdx.x == 0) {
        counts[3 * i] = s0;
        counts[3 * i + 1] = s1;
        counts[3 * i + 2] = s2;
    }
}

void layer_counts(const uint8_t* dist, int64_t n, int N, int delta, int32_t* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_layer_counts, dim3(N), dim3(256), 0, s, dist, n, delta, counts);
    launch_check("layer_counts");
}

// block-wide exclusive scan of a 0/1 flag (256 threads); returns total
__device__ int block_excl_scan(int flag, int* buf, int& excl) {
    const int t = threadIdx.x;
    buf[t] = flag;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = (t >= off) ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    excl = buf[t] - flag;
    const int total = buf[255];
    __syncthreads();
    return total;
}

__global__ void __launch_bounds__(256) k_layer_compact(const uint8_t* dist, int64_t n, int delta, const int64_t* offE,
                                                       const int32_t* counts, int32_t* ext) {
    __shared__ int buf[256];
    const int i = blockIdx.x;
    const uint8_t* di = dist + (int64_t)i * n;
    int32_t* outI = ext + offE[i];
    int32_t* outG = outI + counts[3 * i];
    int32_t* outD = outG + counts[3 * i + 1];
    int b0 = 0, b1 = 0, b2 = 0;
    for (int64_t v0 = 0; v0 < n; v0 += 256) {
        const int64_t v = v0 + threadIdx.x;
        const int d = (v < n) ? di[v] : 255;
        int e0, e1, e2;
        const int t0 = block_excl_scan(d == 0, buf, e0);
        const int t1 = block_excl_scan(d >= 1 && d <= delta, buf, e1);
        const int t2 = block_excl_scan(d == delta + 1, buf, e2);
        if (d == 0) outI[b0 + e0] = (int32_t)v;
        else if (d >= 1 && d <= delta) outG[b1 + e1] = (int32_t)v;
        else if (d == delta + 1) outD[b2 + e2] = (int32_t)v;
        b0 += t0;
        b1 += t1;
        b2 += t2;
    }
}

void layer_compact(const uint8_t* dist, int64_t n, int N, int delta, const int64_t* offE, const int32_t* counts,
                   int32_t* ext, hipStream_t s) {
    hipLaunchKernelGGL(k_layer_compact, dim3(N), dim3(256), 0, s, dist, n, delta, offE, counts, ext);
    launch_check("layer_compact");
}

__global__ void __launch_bounds__(256) k_scan_counts(const int32_t* counts, int64_t n, int64_t* off) {
    __shared__ int64_t buf[256];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t v0 = 0; v0 < n; v0 += 256) {
        const int64_t v = v0 + threadIdx.x;
        const int64_t c = (v < n) ? counts[v] : 0;
        buf[threadIdx.x] = c;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            const int64_t add = (threadIdx.x >= (unsigned)o) ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (v < n) off[v] = carry + buf[threadIdx.x] - c;
        __syncthreads();
        if (threadIdx.x == 255) carry += buf[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[n] = carry;
}

void scan_counts(const int32_t* counts, int64_t n, int64_t* offsets, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(256), 0, s, counts, n, offsets);
    launch_check("scan_counts");
}

__global__ void k_memb_counts(const uint8_t* dist, int64_t n, int N, int delta, int32_t* cnt) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        int c = 0;
        for (int i = 0; i < N; ++i) c += (dist[(int64_t)i * n + g] <= delta);
        cnt[g] = c;
    }
}

void membership_counts(const uint8_t* dist, int64_t n, int N, int delta, int32_t* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_memb_counts, dim3(grid_for(n)), dim3(256), 0, s, dist, n, N, delta, cnt);
    launch_check("memb_counts");
}

__device__ int lower_bound_i32(const int32_t* a, int len, int32_t x) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// local index of global g inside Omega~_i given its layer value
__device__ __forceinline__ int local_index(const int32_t* exti, const int32_t* cnt3, int d, int delta, int32_t g) {
    const int nI = cnt3[0], nG = cnt3[1], nD = cnt3[2];
    if (d == 0) return lower_bound_i32(exti, nI, g);
    if (d <= delta) return nI + lower_bound_i32(exti + nI, nG, g);
    return nI + nG + lower_bound_i32(exti + nI + nG, nD, g);
}

__global__ void k_memb_fill(const uint8_t* dist, int64_t n, int N, int delta, const int64_t* offE, const int64_t* offO,
                            const int32_t* counts, const int32_t* ext, const int64_t* memb_ptr, int64_t* memb) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        int64_t pos = memb_ptr[g];
        for (int i = 0; i < N; ++i) {
            const int d = dist[(int64_t)i * n + g];
            if (d <= delta) memb[pos++] = offO[i] + local_index(ext + offE[i], counts + 3 * i, d, delta, (int32_t)g);
        }
    }
}

void membership_fill(const uint8_t* dist, int64_t n, int N, int delta, const int64_t* offE, const int64_t* offO,
                     const int32_t* counts, const int32_t* ext, const int64_t* memb_ptr, int64_t* memb,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_memb_fill, dim3(grid_for(n)), dim3(256), 0, s, dist, n, N, delta, offE, offO, counts, ext,
                       memb_ptr, memb);
    launch_check("memb_fill");
}

// one block per subdomain
__global__ void k_omega_flatten(const int64_t* offE, const int64_t* offO, const int32_t* counts, const int32_t* ext,
                                int32_t* omega_flat, int32_t* ilocal) {
    const int i = blockIdx.x;
    const int nI = counts[3 * i], ni = nI + counts[3 * i + 1];
    const int32_t* e = ext + offE[i];
    for (int r = threadIdx.x; r < ni; r += blockDim.x) {
        omega_flat[offO[i] + r] = e[r];
        if (r < nI) ilocal[e[r]] = r;
    }
}

void omega_flatten(int N, const int64_t* offE, const int64_t* offO, const int32_t* counts, const int32_t* ext,
                   int64_t, int32_t* omega_flat, int32_t* ilocal, hipStream_t s) {
    hipLaunchKernelGGL(k_omega_flatten, dim3(N), dim3(256), 0, s, offE, offO, counts, ext, omega_flat, ilocal);
    launch_check("omega_flatten");
}

// ===========================================================================
// Extraction of dense X_i^T and A_ii (3.1), one thread per local row
// ===========================================================================
__global__ void k_extract(CsrDev A, int N, int delta, int64_t n, const uint8_t* dist, const int64_t* offE,
                          const int64_t* offO, const int32_t* counts, const int32_t* ext, double* const* Y,
                          double* const* Aii, int64_t total) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        // subdomain i with offO[i] <= q < offO[i+1]
        int lo = 0, hi = N;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offO[mid] <= q) lo = mid; else hi = mid;
        }
        const int i = lo;
        const int r = (int)(q - offO[i]);
        const int32_t* cnt3 = counts + 3 * i;
        const int ni = cnt3[0] + cnt3[1];
        const int nt = ni + cnt3[2];
        const int32_t* exti = ext + offE[i];
        const int32_t g = exti[r];
        const uint8_t* di = dist + (int64_t)i * n;
        double* Yi = Y[i];
        double* Ai = Aii[i];
        for (int e = A.rowptr[g]; e < A.rowptr[g + 1]; ++e) {
            const int32_t c = A.colind[e];
            const int d = di[c];
            if (d > delta + 1) continue;  // cannot happen for rows of Omega_i (kept for safety)
            const int lc = local_index(exti, cnt3, d, delta, c);
            const double a = A.val[e];
            Yi[lc + (int64_t)r * nt] = a;       // Y = X^T: Y(lc, r) = X(r, lc)
            if (lc < ni) Ai[r + (int64_t)lc * ni] = a;
        }
    }
}

void extract(const CsrDev& A, int N, int delta, int64_t n, const uint8_t* dist, const int64_t* offE,
             const int64_t* offO, const int32_t* counts, const int32_t* ext, double* const* Y, double* const* Aii,
             int64_t total_rows, hipStream_t s) {
    hipLaunchKernelGGL(k_extract, dim3(grid_for(total_rows)), dim3(256), 0, s, A, N, delta, n, dist, offE, offO,
                       counts, ext, Y, Aii, total_rows);
    launch_check("extract");
}

// ===========================================================================
// vectors
// ===========================================================================
// 8 lanes per row, column-major multi-RHS: each matrix entry is read once for
// up to 8 right-hand sides; every column is summed in the same order as a
// single right-hand side, so each column's result does not depend on nrhs
__global__ void k_spmv(CsrDev A, const double* x, double* y, int nrhs) {
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t row = gt >> 3;
    const int sub = threadIdx.x & 7;
    if (row >= A.n) return;
    const int b = A.rowptr[row], e = A.rowptr[row + 1];
    for (int k0 = 0; k0 < nrhs; k0 += 8) {
        const int kn = min(8, nrhs - k0);
        const double* xk = x + (int64_t)k0 * A.n;
        double s[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] = 0.0;
        for (int q = b + sub; q < e; q += 8) {
            const double a = A.val[q];
            const int64_t c = A.colind[q];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < kn) s[k] += a * xk[c + (int64_t)k * A.n];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            double v = s[k];
            v += __shfl_xor(v, 1, 8);
            v += __shfl_xor(v, 2, 8);
            v += __shfl_xor(v, 4, 8);
            if (sub == 0 && k < kn) y[row + (int64_t)(k0 + k) * A.n] = v;
        }
    }
}

void spmv(const CsrDev& A, const double* x, double* y, int nrhs, hipStream_t s) {
    const int64_t threads = A.n * 8;
    hipLaunchKernelGGL(k_spmv, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, A, x, y, nrhs);
    launch_check("spmv");
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
void fill(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
    launch_check("fill");
}

constexpr int kDotBlocks = 512;
__global__ void k_dot_part(const double* x, const double* y, int64_t n, double* partial) {
    __shared__ double red[4];
    const int k = blockIdx.y;
    const double* xk = x + (int64_t)k * n;
    const double* yk = y + (int64_t)k * n;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += xk[i] * yk[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[k * kDotBlocks + blockIdx.x] = s;
}
__global__ void k_dot_final(const double* partial, double* out) {
    __shared__ double red[4];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < kDotBlocks; i += blockDim.x) s += partial[k * kDotBlocks + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[k] = s;
}
__global__ void k_dot_seg_part(const double* x, const double* y, const int64_t* off, double* partial) {
    __shared__ double red[4];
    const int k = blockIdx.y;
    const int64_t b = off[k], e = off[k + 1];
    double s = 0.0;
    for (int64_t i = b + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < e; i += (int64_t)gridDim.x * blockDim.x)
        s += x[i] * y[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[k * kDotBlocks + blockIdx.x] = s;
}
void dot_seg(const double* x, const double* y, const int64_t* off, int nseg, double* partial, double* out,
             hipStream_t s) {
    hipLaunchKernelGGL(k_dot_seg_part, dim3(kDotBlocks, nseg), dim3(256), 0, s, x, y, off, partial);
    hipLaunchKernelGGL(k_dot_final, dim3(nseg), dim3(256), 0, s, partial, out);
    launch_check("dot_seg");
}
void dot(const double* x, const double* y, int64_t n, int nrhs, double* partial, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_part, dim3(kDotBlocks, nrhs), dim3(256), 0, s, x, y, n, partial);
    hipLaunchKernelGGL(k_dot_final, dim3(nrhs), dim3(256), 0, s, partial, out);
    launch_check("dot");
}

__global__ void k_gather(const double* x, const int32_t* idx, int64_t m, double* out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = x[idx[i]];
}
void gather(const double* x, const int32_t* idx, int64_t m, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather, dim3(grid_for(m)), dim3(256), 0, s, x, idx, m, out);
    launch_check("gather");
}

__global__ void k_scatter_sum(const double* loc, const int64_t* mp, const int64_t* memb, int64_t n, double* z, int acc) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        double s = acc ? z[g] : 0.0;
        for (int64_t q = mp[g]; q < mp[g + 1]; ++q) s += loc[memb[q]];
        z[g] = s;
    }
}
void scatter_sum(const double* loc, const int64_t* memb_ptr, const int64_t* memb, int64_t n, double* z,
                 bool accumulate, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_sum, dim3(grid_for(n)), dim3(256), 0, s, loc, memb_ptr, memb, n, z, accumulate ? 1 : 0);
    launch_check("scatter_sum");
}

}  // namespace dd
