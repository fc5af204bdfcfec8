// Coarse space assembly and transfer kernels.
#include "coarse.hpp"

#include <algorithm>

namespace dd {

// one thread per subdomain j: count rows of Omega_j by owner
__global__ void k_pair_counts(SubInfo S, int32_t* cnt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S.N) return;
    const int nI = S.counts[3 * j], ni = nI + S.counts[3 * j + 1];
    const int32_t* e = S.ext + S.offE[j];
    int32_t* row = cnt + (int64_t)j * S.N;
    row[j] += nI;
    for (int r = nI; r < ni; ++r) row[S.part[e[r]]] += 1;
}

void pair_counts(const SubInfo& S, int32_t* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_counts, dim3((S.N + 63) / 64), dim3(64), 0, s, S, cnt);
    launch_check("pair_counts");
}

// rows of Omega_j grouped by owner, in local order (deterministic)
__global__ void k_pair_fill(SubInfo S, const int64_t* pairoff, int32_t* cursor, int32_t* zr, int32_t* pr) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= S.N) return;
    const int nI = S.counts[3 * j], ni = nI + S.counts[3 * j + 1];
    const int32_t* e = S.ext + S.offE[j];
    for (int r = 0; r < ni; ++r) {
        const int32_t g = e[r];
        const int o = S.part[g];
        const int64_t key = (int64_t)j * S.N + o;
        const int64_t pos = pairoff[key] + cursor[key]++;
        zr[pos] = S.ilocal[g];
        pr[pos] = r;
    }
}

void pair_fill(const SubInfo& S, const int64_t* pairoff, int32_t* cursor, int32_t* zr, int32_t* pr, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_fill, dim3((S.N + 63) / 64), dim3(64), 0, s, S, pairoff, cursor, zr, pr);
    launch_check("pair_fill");
}

// P_j(r, a) = sum over stored A(g, c), c in Omega_Ij, of A(g,c) Z_j(ilocal(c), a), g = Omega_j[r]
struct OpBuildP {
    CsrDev A;
    SubInfo S;
    double* const* P;
    __device__ int tiles(int j) const {
        const int ni = S.counts[3 * j] + S.counts[3 * j + 1];
        return (S.pcnt[j] > 0) ? (ni + 63) / 64 : 0;
    }
    __device__ void operator()(int j, int t) const {
        const int nI = S.counts[3 * j], ni = nI + S.counts[3 * j + 1];
        const int p = S.pcnt[j];
        const int32_t* e = S.ext + S.offE[j];
        const double* Zj = S.Z[j];
        double* Pj = P[j];
        for (int q = threadIdx.x; q < 64 * p; q += blockDim.x) {
            const int r = t * 64 + (q & 63), a = q >> 6;
            if (r >= ni) continue;
            const int32_t g = e[r];
            double sum = 0.0;
            for (int k = A.rowptr[g]; k < A.rowptr[g + 1]; ++k) {
                const int32_t c = A.colind[k];
                if (S.part[c] == j) sum += A.val[k] * Zj[S.ilocal[c] + (int64_t)a * nI];
            }
            Pj[r + (int64_t)a * ni] = sum;
        }
    }
};

void build_p(const CsrDev& A, const SubInfo& S, double* const* P, const std::vector<int>& hni,
             const std::vector<int>& hp, hipStream_t s) {
    int64_t tot = 0;
    for (int j = 0; j < S.N; ++j)
        if (hp[j] > 0) tot += ceil_div(hni[j], 64);
    launch_tiles(OpBuildP{A, S, P}, S.N, tot, s, "build_p");
}

struct OpEBlock {
    SubInfo S;
    const PairItem* pairs;
    double* const* P;
    const int32_t* zr;
    const int32_t* pr;
    __device__ int tiles(int q) const {
        const PairItem& pi = pairs[q];
        return ((S.pcnt[pi.i] + 63) / 64) * ((S.pcnt[pi.j] + 63) / 64);
    }
    __device__ void operator()(int q, int t) const {
        __shared__ TileSmem sm;
        const PairItem pi = pairs[q];
        const int p_i = S.pcnt[pi.i], p_j = S.pcnt[pi.j];
        const int tm = (p_i + 63) / 64;
        const int i0 = (t % tm) * 64, j0 = (t / tm) * 64;
        const int nIi = S.counts[3 * pi.i];
        const int nj = S.counts[3 * pi.j] + S.counts[3 * pi.j + 1];
        double4_t acc[2][2];
        acc_zero(acc);
        mfma_tile_64<true, false>(S.Z[pi.i], nIi, P[pi.j], nj, p_i, p_j, pi.nrows, i0, j0, sm, acc,
                                  zr + pi.rows, pr + pi.rows);
        double* Eb = pi.out;
        const int64_t ld = pi.ldo;
        acc_foreach(acc, [&](int r, int c, double v) {
            const int gi = i0 + r, gj = j0 + c;
            if (gi < p_i && gj < p_j) Eb[gi + gj * ld] = v;
        });
    }
};

void assemble_e(const SubInfo& S, const PairItem* dpairs, const std::vector<PairItem>& hpairs,
                const std::vector<int>& hp, double* const* P, const int32_t* zr, const int32_t* pr, hipStream_t s) {
    int64_t tot = 0;
    for (auto& q : hpairs) tot += (int64_t)ceil_div(hp[q.i], 64) * ceil_div(hp[q.j], 64);
    launch_tiles(OpEBlock{S, dpairs, P, zr, pr}, (int)hpairs.size(), tot, s, "assemble_e");
}

__global__ void k_block_adj(CsrDev A, const int32_t* part, int N, uint8_t* adj) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < A.n; u += (int64_t)gridDim.x * blockDim.x) {
        const int pu = part[u];
        for (int e = A.rowptr[u]; e < A.rowptr[u + 1]; ++e) {
            const int pv = part[A.colind[e]];
            if (pv != pu) adj[(int64_t)pu * N + pv] = 1;  // every writer stores the same value
        }
    }
}

void block_adjacency(const CsrDev& A, const int32_t* part, int N, uint8_t* adj, hipStream_t s) {
    hipLaunchKernelGGL(k_block_adj, dim3((unsigned)std::min<int64_t>((A.n + 255) / 256, 65536)), dim3(256), 0, s, A,
                       part, N, adj);
    launch_check("block_adjacency");
}

// one block per coarse dof (i, a)
__global__ void k_restrict(SubInfo S, int64_t nC, const double* x, double* y) {
    __shared__ double red[4];
    for (int64_t q = blockIdx.x; q < nC; q += gridDim.x) {
        int lo = 0, hi = S.N;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (S.offC[mid] <= q) lo = mid; else hi = mid;
        }
        const int i = lo;
        const int a = (int)(q - S.offC[i]);
        const int nI = S.counts[3 * i];
        const double* z = S.Z[i] + (int64_t)a * nI;
        const int32_t* I = S.ext + S.offE[i];
        double sum = 0.0;
        for (int r = threadIdx.x; r < nI; r += blockDim.x) sum += z[r] * x[I[r]];
        sum = block_sum(sum, red);
        if (threadIdx.x == 0) y[q] = sum;
        __syncthreads();
    }
}

void restrict_coarse(const SubInfo& S, int64_t nC, const double* x, double* y, hipStream_t s) {
    if (nC <= 0) return;
    hipLaunchKernelGGL(k_restrict, dim3((unsigned)std::min<int64_t>(nC, 65536)), dim3(256), 0, s, S, nC, x, y);
    launch_check("restrict");
}

// one thread per fine interior node: node g = I_i[r]
__global__ void k_prolong(SubInfo S, int64_t total, const int64_t* offI, const double* y, double* z) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = S.N;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (offI[mid] <= q) lo = mid; else hi = mid;
        }
        const int i = lo;
        const int r = (int)(q - offI[i]);
        const int nI = S.counts[3 * i];
        const int p = S.pcnt[i];
        const double* Zi = S.Z[i];
        const double* yi = y + S.offC[i];
        double sum = 0.0;
        for (int a = 0; a < p; ++a) sum += Zi[r + (int64_t)a * nI] * yi[a];
        z[S.ext[S.offE[i] + r]] += sum;
    }
}

void prolong_coarse(const SubInfo& S, const int64_t* offI, int64_t nI_total, const double* y, double* z, hipStream_t s) {
    if (nI_total <= 0) return;
    hipLaunchKernelGGL(k_prolong, dim3((unsigned)std::min<int64_t>((nI_total + 255) / 256, 65536)), dim3(256), 0, s, S,
                       nI_total, offI, y, z);
    launch_check("prolong");
}

}  // namespace dd
