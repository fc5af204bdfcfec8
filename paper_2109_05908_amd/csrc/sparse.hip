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
// Overlap sets by frontier lists (Sec. 2).  Omega_i grows from the part I_i
// by delta layers of A's graph and Delta_i is the next layer.  Every list is
// one ascending segment per subdomain of a flat int32 buffer, so memory and
// work are proportional to the sizes of the sets times their row lengths,
// whatever the number of subdomains.
// ===========================================================================

// block-wide exclusive scan of an int value (256 threads); returns the total
__device__ int block_excl_scan(int v, int* buf, int& excl) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = (t >= off) ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    excl = buf[t] - v;
    const int total = buf[255];
    __syncthreads();
    return total;
}

__device__ int lower_bound_i32(const int32_t* a, int len, int32_t x) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool seg_has(const int32_t* a, int len, int32_t x) {
    const int p = lower_bound_i32(a, len, x);
    return p < len && a[p] == x;
}

// Ascending sort of a[0, len) by one workgroup.  Bitonic network in the form
// whose first comparator stage of every merge pairs mirrored positions: all
// comparators then point upwards, so positions at or past len behave as
// +infinity and their comparators are skipped (any length, no padding).
__device__ void wg_sort(int32_t* a, int64_t len) {
    int64_t P = 1;
    while (P < len) P <<= 1;
    for (int64_t k = 2; k <= P; k <<= 1) {
        const int64_t h = k >> 1;
        for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
            const int64_t i = (t / h) * k + (t % h);
            const int64_t l = i ^ (k - 1);
            if (l < len) {
                const int32_t x = a[i], y = a[l];
                if (x > y) { a[i] = y; a[l] = x; }
            }
        }
        __syncthreads();
        for (int64_t j = h >> 1; j > 0; j >>= 1) {
            for (int64_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const int64_t i = (t / j) * 2 * j + (t % j);
                const int64_t l = i + j;
                if (l < len) {
                    const int32_t x = a[i], y = a[l];
                    if (x > y) { a[i] = y; a[l] = x; }
                }
            }
            __syncthreads();
        }
    }
}

constexpr int kSortLds = 8192;

// merges the ascending runs x[0, na) and y[0, nb) into out[0, na + nb), one
// workgroup: every thread finds its share of the output by a binary search on
// its diagonal (merge path) and merges that share sequentially
__device__ void wg_merge(const int32_t* x, int64_t na, const int32_t* y, int64_t nb, int32_t* out) {
    const int64_t m = na + nb;
    const int64_t per = (m + blockDim.x - 1) / blockDim.x;
    const int64_t d0 = min(m, (int64_t)threadIdx.x * per), d1 = min(m, d0 + per);
    if (d0 >= d1) return;
    // i = number taken from x among the first d0 outputs
    int64_t lo = max((int64_t)0, d0 - nb), hi = min(d0, na);
    while (lo < hi) {
        const int64_t i = (lo + hi) >> 1;
        if (x[i] < y[d0 - i - 1]) lo = i + 1; else hi = i;
    }
    int64_t i = lo, j = d0 - lo;
    for (int64_t d = d0; d < d1; ++d) {
        if (j >= nb || (i < na && x[i] <= y[j])) out[d] = x[i++];
        else out[d] = y[j++];
    }
}

// sorts data[beg[i], end[i]) ascending, one workgroup per segment: in LDS when
// it fits, else LDS-sized runs merged pairwise through tmp (same offsets)
__global__ void __launch_bounds__(256) k_seg_sort(int32_t* data, int32_t* tmp, const int64_t* beg,
                                                  const int64_t* end) {
    __shared__ int32_t sm[kSortLds];
    const int i = blockIdx.x;
    int32_t* a = data + beg[i];
    const int64_t len = end[i] - beg[i];
    if (len < 2) return;
    for (int64_t c0 = 0; c0 < len; c0 += kSortLds) {
        const int64_t cl = min((int64_t)kSortLds, len - c0);
        for (int64_t p = threadIdx.x; p < cl; p += blockDim.x) sm[p] = a[c0 + p];
        __syncthreads();
        wg_sort(sm, cl);
        for (int64_t p = threadIdx.x; p < cl; p += blockDim.x) a[c0 + p] = sm[p];
        __syncthreads();
    }
    if (len <= kSortLds) return;
    int32_t* src = a;
    int32_t* dst = tmp + beg[i];
    for (int64_t w = kSortLds; w < len; w *= 2) {
        for (int64_t x0 = 0; x0 < len; x0 += 2 * w) {
            const int64_t na = min(w, len - x0);
            const int64_t nb = min(w, len - x0 - na);
            wg_merge(src + x0, na, src + x0 + na, nb, dst + x0);
        }
        __syncthreads();
        int32_t* t = src; src = dst; dst = t;
    }
    if (src != a)
        for (int64_t p = threadIdx.x; p < len; p += blockDim.x) a[p] = src[p];
}

// tmp: scratch of the same extent as data (used only by segments longer than kSortLds)
static void seg_sort(int32_t* data, int32_t* tmp, const int64_t* beg, const int64_t* end, int nseg,
                     hipStream_t s) {
    if (nseg > 0) hipLaunchKernelGGL(k_seg_sort, dim3(nseg), dim3(256), 0, s, data, tmp, beg, end);
    launch_check("seg_sort");
}

__global__ void k_part_hist(const int32_t* part, int64_t n, int32_t* cnt) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[part[v]], 1);
}

__global__ void k_part_place(const int32_t* part, int64_t n, const int64_t* off, int32_t* cursor, int32_t* L) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int i = part[v];
        L[off[i] + atomicAdd(&cursor[i], 1)] = (int32_t)v;
    }
}

// a neighbour of a vertex at distance k-1 is at distance k-2, k-1 or k: the
// candidates of layer k are the neighbours of layer k-1 (L1) found neither in
// L1 nor in layer k-2 (L2, may be null)
struct Frontier {
    const int32_t* L1;
    const int64_t* off1;
    const int32_t* L2;
    const int64_t* off2;
    __device__ bool fresh(int i, int32_t c) const {
        if (seg_has(L1 + off1[i], (int)(off1[i + 1] - off1[i]), c)) return false;
        return !(L2 && seg_has(L2 + off2[i], (int)(off2[i + 1] - off2[i]), c));
    }
};

// cnt[i] = number of candidate entries (with repeats) of subdomain i
__global__ void __launch_bounds__(256) k_front_len(CsrDev A, Frontier F, int64_t* cnt) {
    __shared__ int64_t red[256];
    const int i = blockIdx.x;
    int64_t acc = 0;
    for (int64_t p = F.off1[i] + threadIdx.x; p < F.off1[i + 1]; p += blockDim.x) {
        const int32_t u = F.L1[p];
        for (int q = A.rowptr[u]; q < A.rowptr[u + 1]; ++q) acc += F.fresh(i, A.colind[q]);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[i] = red[0];
}

// cand[coff[i] ...] = the candidate entries, in frontier and row order
__global__ void __launch_bounds__(256) k_front_fill(CsrDev A, Frontier F, const int64_t* coff, int32_t* cand) {
    __shared__ int buf[256];
    const int i = blockIdx.x;
    int64_t base = coff[i];
    for (int64_t p0 = F.off1[i]; p0 < F.off1[i + 1]; p0 += 256) {
        const int64_t p = p0 + threadIdx.x;
        int cnt = 0, r0 = 0, r1 = 0;
        if (p < F.off1[i + 1]) {
            const int32_t u = F.L1[p];
            r0 = A.rowptr[u];
            r1 = A.rowptr[u + 1];
            for (int q = r0; q < r1; ++q) cnt += F.fresh(i, A.colind[q]);
        }
        int e;
        const int tot = block_excl_scan(cnt, buf, e);
        for (int q = r0; q < r1; ++q) {
            const int32_t c = A.colind[q];
            if (F.fresh(i, c)) cand[base + e++] = c;
        }
        base += tot;
    }
}

// In place on each sorted candidate segment: keep the first copy of every
// vertex; kept[i] = the new length
__global__ void __launch_bounds__(256) k_front_unique(int32_t* cand, const int64_t* coff, int32_t* kept) {
    __shared__ int buf[256];
    __shared__ int32_t lastv;
    const int i = blockIdx.x;
    int32_t* c = cand + coff[i];
    const int64_t len = coff[i + 1] - coff[i];
    int64_t base = 0;
    for (int64_t p0 = 0; p0 < len; p0 += 256) {
        const int64_t p = p0 + threadIdx.x;
        int32_t x = 0;
        int keep = 0;
        if (p < len) {
            x = c[p];
            keep = (p == 0) || ((threadIdx.x > 0 ? c[p - 1] : lastv) != x);
        }
        __syncthreads();  // every read of this chunk (and of lastv) is done
        if (threadIdx.x == 255) lastv = x;
        int e;
        const int tot = block_excl_scan(keep, buf, e);  // writes land below p0 + 256, reads come from above
        if (keep) c[base + e] = x;
        base += tot;
    }
    if (threadIdx.x == 0) kept[i] = (int32_t)base;
}

// dst[dbeg[i] + r] = src[sbeg[i] + r] for r < loff[i+1] - loff[i]
__global__ void k_seg_place(const int32_t* src, const int64_t* sbeg, const int64_t* loff, const int64_t* dbeg,
                            int32_t* dst) {
    const int i = blockIdx.x;
    const int64_t len = loff[i + 1] - loff[i];
    for (int64_t r = threadIdx.x; r < len; r += blockDim.x) dst[dbeg[i] + r] = src[sbeg[i] + r];
}

namespace {
// one list per subdomain: flat buffer plus host and device offsets
struct SegLists {
    DBuf<int32_t> v;
    std::vector<int64_t> hoff;
    DBuf<int64_t> off;
    int64_t len(int i) const { return hoff[i + 1] - hoff[i]; }
};

std::vector<int64_t> prefix(const std::vector<int64_t>& c) {
    std::vector<int64_t> o(c.size() + 1, 0);
    for (size_t i = 0; i < c.size(); ++i) o[i + 1] = o[i] + c[i];
    return o;
}
}  // namespace

void overlap_sets(const CsrDev& A, const int32_t* part, int N, int delta, std::vector<int32_t>& hcounts,
                  DBuf<int32_t>& ext, hipStream_t s) {
    const int64_t n = A.n;
    std::vector<SegLists> L(delta + 2);
    // layer 0: the part of every subdomain, ascending
    {
        DBuf<int32_t> cnt(N), cur(N);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(N)), dim3(256), 0, s, cnt.p, (int64_t)N, 0);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(N)), dim3(256), 0, s, cur.p, (int64_t)N, 0);
        hipLaunchKernelGGL(k_part_hist, dim3(grid_for(n)), dim3(256), 0, s, part, n, cnt.p);
        std::vector<int32_t> h(N);
        d2h(h.data(), cnt.p, N, s);
        DD_HIP(hipStreamSynchronize(s));
        L[0].hoff = prefix(std::vector<int64_t>(h.begin(), h.end()));
        L[0].off = upload(L[0].hoff, s);
        L[0].v.alloc(n);
        hipLaunchKernelGGL(k_part_place, dim3(grid_for(n)), dim3(256), 0, s, part, n, L[0].off.p, cur.p, L[0].v.p);
        DBuf<int32_t> tmp(n);
        seg_sort(L[0].v.p, tmp.p, L[0].off.p, L[0].off.p + 1, N, s);
        DD_HIP(hipStreamSynchronize(s));  // tmp is released here
    }
    // layer k: the neighbours of layer k-1 outside layers k-1 and k-2
    for (int k = 1; k <= delta + 1; ++k) {
        const SegLists* G = (k >= 2) ? &L[k - 2] : nullptr;
        const Frontier F{L[k - 1].v.p, L[k - 1].off.p, G ? G->v.p : nullptr, G ? G->off.p : nullptr};
        DBuf<int64_t> cl(N);
        hipLaunchKernelGGL(k_front_len, dim3(N), dim3(256), 0, s, A, F, cl.p);
        std::vector<int64_t> hc(N);
        d2h(hc.data(), cl.p, N, s);
        DD_HIP(hipStreamSynchronize(s));
        const std::vector<int64_t> hcoff = prefix(hc);
        DBuf<int64_t> coff = upload(hcoff, s);
        DBuf<int32_t> cand(hcoff[N]), tmp(hcoff[N]);
        hipLaunchKernelGGL(k_front_fill, dim3(N), dim3(256), 0, s, A, F, coff.p, cand.p);
        seg_sort(cand.p, tmp.p, coff.p, coff.p + 1, N, s);
        DBuf<int32_t> kept(N);
        hipLaunchKernelGGL(k_front_unique, dim3(N), dim3(256), 0, s, cand.p, coff.p, kept.p);
        std::vector<int32_t> hk(N);
        d2h(hk.data(), kept.p, N, s);
        DD_HIP(hipStreamSynchronize(s));
        L[k].hoff = prefix(std::vector<int64_t>(hk.begin(), hk.end()));
        L[k].off = upload(L[k].hoff, s);
        L[k].v.alloc(L[k].hoff[N]);
        hipLaunchKernelGGL(k_seg_place, dim3(N), dim3(256), 0, s, cand.p, coff.p, L[k].off.p, L[k].off.p,
                           L[k].v.p);
        DD_HIP(hipStreamSynchronize(s));  // cand, tmp and coff are released on return
    }
    launch_check("overlap layers");

    // ext[offE[i] ...] = [I_i, Gamma_i (layers 1..delta merged), Delta_i (layer delta+1)]
    hcounts.assign(3 * (size_t)N, 0);
    std::vector<int64_t> offE(N + 1, 0);
    for (int i = 0; i < N; ++i) {
        int64_t g = 0;
        for (int k = 1; k <= delta; ++k) g += L[k].len(i);
        hcounts[3 * i] = (int32_t)L[0].len(i);
        hcounts[3 * i + 1] = (int32_t)g;
        hcounts[3 * i + 2] = (int32_t)L[delta + 1].len(i);
        offE[i + 1] = offE[i] + L[0].len(i) + g + L[delta + 1].len(i);
    }
    ext.alloc(offE[N]);
    std::vector<int64_t> dst(N), gbeg(N), gend(N);
    for (int k = 0; k <= delta + 1; ++k) {
        for (int i = 0; i < N; ++i) {
            int64_t at = offE[i];
            for (int q = 0; q < k; ++q) at += L[q].len(i);
            dst[i] = at;
        }
        DBuf<int64_t> ddst = upload(dst, s);
        hipLaunchKernelGGL(k_seg_place, dim3(N), dim3(256), 0, s, L[k].v.p, L[k].off.p, L[k].off.p, ddst.p,
                           ext.p);
        DD_HIP(hipStreamSynchronize(s));
    }
    if (delta >= 2) {  // Gamma_i gathers several ascending layers
        for (int i = 0; i < N; ++i) {
            gbeg[i] = offE[i] + hcounts[3 * i];
            gend[i] = gbeg[i] + hcounts[3 * i + 1];
        }
        DBuf<int64_t> db = upload(gbeg, s), de = upload(gend, s);
        DBuf<int32_t> tmp(offE[N]);
        seg_sort(ext.p, tmp.p, db.p, de.p, N, s);
        DD_HIP(hipStreamSynchronize(s));
    }
    launch_check("overlap sets");
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

// cnt[g] += 1 for every g of Omega_i = I_i u Gamma_i, one workgroup per subdomain
__global__ void k_memb_count(const int64_t* offE, const int32_t* counts, const int32_t* ext, int32_t* cnt) {
    const int i = blockIdx.x;
    const int ni = counts[3 * i] + counts[3 * i + 1];
    for (int r = threadIdx.x; r < ni; r += blockDim.x) atomicAdd(&cnt[ext[offE[i] + r]], 1);
}

__global__ void k_memb_place(const int64_t* offE, const int64_t* offO, const int32_t* counts, const int32_t* ext,
                             const int64_t* memb_ptr, int32_t* cursor, int64_t* memb) {
    const int i = blockIdx.x;
    const int ni = counts[3 * i] + counts[3 * i + 1];
    for (int r = threadIdx.x; r < ni; r += blockDim.x) {
        const int32_t g = ext[offE[i] + r];
        memb[memb_ptr[g] + atomicAdd(&cursor[g], 1)] = offO[i] + r;
    }
}

// every node's list ascending (heap sort per thread); positions grow with the
// subdomain index, so this is subdomain order
__global__ void k_memb_sort(const int64_t* memb_ptr, int64_t n, int64_t* memb) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        int64_t* a = memb + memb_ptr[g];
        const int64_t m = memb_ptr[g + 1] - memb_ptr[g];
        auto sift = [a](int64_t r, int64_t end) {
            while (2 * r + 1 < end) {
                int64_t c = 2 * r + 1;
                if (c + 1 < end && a[c] < a[c + 1]) ++c;
                if (a[r] >= a[c]) return;
                const int64_t t = a[r]; a[r] = a[c]; a[c] = t;
                r = c;
            }
        };
        for (int64_t r = m / 2 - 1; r >= 0; --r) sift(r, m);
        for (int64_t end = m - 1; end > 0; --end) {
            const int64_t t = a[0]; a[0] = a[end]; a[end] = t;
            sift(0, end);
        }
    }
}

void membership(const int64_t* offE, const int64_t* offO, const int32_t* counts, const int32_t* ext, int N,
                int64_t n, DBuf<int64_t>& memb_ptr, DBuf<int64_t>& memb, int64_t total, hipStream_t s) {
    DBuf<int32_t> cnt(n);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, cnt.p, n, 0);
    hipLaunchKernelGGL(k_memb_count, dim3(N), dim3(256), 0, s, offE, counts, ext, cnt.p);
    memb_ptr.alloc(n + 1);
    scan_counts(cnt.p, n, memb_ptr.p, s);
    memb.alloc(total);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, cnt.p, n, 0);
    hipLaunchKernelGGL(k_memb_place, dim3(N), dim3(256), 0, s, offE, offO, counts, ext, memb_ptr.p, cnt.p, memb.p);
    hipLaunchKernelGGL(k_memb_sort, dim3(grid_for(n)), dim3(256), 0, s, memb_ptr.p, n, memb.p);
    DD_HIP(hipStreamSynchronize(s));  // cnt is released on return
    launch_check("membership");
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

// local index of g in Omega~_i = [I_i, Gamma_i, Delta_i] (each ascending), -1 if absent
__device__ __forceinline__ int local_index(const int32_t* exti, const int32_t* cnt3, int32_t g) {
    const int nI = cnt3[0], nG = cnt3[1], nD = cnt3[2];
    int p = lower_bound_i32(exti, nI, g);
    if (p < nI && exti[p] == g) return p;
    p = lower_bound_i32(exti + nI, nG, g);
    if (p < nG && exti[nI + p] == g) return nI + p;
    p = lower_bound_i32(exti + nI + nG, nD, g);
    if (p < nD && exti[nI + nG + p] == g) return nI + nG + p;
    return -1;
}

// ===========================================================================
// Extraction of dense X_i^T and A_ii (3.1), one thread per local row
// ===========================================================================
__global__ void k_extract(CsrDev A, int N, const int64_t* offE, const int64_t* offO, const int32_t* counts,
                          const int32_t* ext, double* const* Y, double* const* Aii, int64_t total) {
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
        double* Yi = Y[i];
        double* Ai = Aii[i];
        for (int e = A.rowptr[g]; e < A.rowptr[g + 1]; ++e) {
            const int lc = local_index(exti, cnt3, A.colind[e]);
            if (lc < 0) continue;  // cannot happen for rows of Omega_i (kept for safety)
            const double a = A.val[e];
            Yi[lc + (int64_t)r * nt] = a;       // Y = X^T: Y(lc, r) = X(r, lc)
            if (lc < ni) Ai[r + (int64_t)lc * ni] = a;
        }
    }
}

void extract(const CsrDev& A, int N, const int64_t* offE, const int64_t* offO, const int32_t* counts,
             const int32_t* ext, double* const* Y, double* const* Aii, int64_t total_rows, hipStream_t s) {
    hipLaunchKernelGGL(k_extract, dim3(grid_for(total_rows)), dim3(256), 0, s, A, N, offE, offO, counts, ext, Y, Aii,
                       total_rows);
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
