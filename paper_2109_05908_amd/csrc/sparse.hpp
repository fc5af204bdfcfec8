// Graph, index-map, extraction and vector kernels (integer parts bit-exact).
#pragma once
#include "common.hpp"

#include <vector>

namespace dd {

struct CsrDev {
    int64_t n = 0, nnz = 0;
    const int32_t* rowptr = nullptr;
    const int32_t* colind = nullptr;
    const double* val = nullptr;
};

// --- partition (seeded greedy graph growing) ---
void ggg_partition(const CsrDev& A, int N, uint64_t seed, int32_t* part, hipStream_t s);
// the same without allocating: work arrays in a file-scope device array of
// kGggMaxN + kGggMaxParts + 64 int32 per GPU (n <= kGggMaxN, N <= kGggMaxParts)
constexpr int64_t kGggMaxN = (int64_t)1 << 22;
constexpr int kGggMaxParts = 1 << 16;
void ggg_partition_noalloc(const CsrDev& A, int N, uint64_t seed, int32_t* part, hipStream_t s);

// --- validation: every id in [0, N); counts per part (device int32[N]) ---
int validate_partition(const int32_t* part, int64_t n, int N, int32_t* dcounts, hipStream_t s);

// --- overlap sets by frontier lists (one ascending segment per subdomain) ---
// hcounts[3*i + {0,1,2}] = |I_i|, |Gamma_i|, |Delta_i| (host); ext (allocated
// here) holds [I_i, Gamma_i, Delta_i], each ascending, at offsets that are the
// prefix sums of the three counts.
void overlap_sets(const CsrDev& A, const int32_t* part, int N, int delta, std::vector<int32_t>& hcounts,
                  DBuf<int32_t>& ext, hipStream_t s);

// Exclusive prefix sum of int32 counts into int64 offsets (n+1 entries), one workgroup.
void scan_counts(const int32_t* counts, int64_t n, int64_t* offsets, hipStream_t s);

// Membership of every node: memb_ptr[g]..memb_ptr[g+1] lists positions (in the
// concatenated Omega buffer, offO[i] + local index) of the subdomains containing g,
// in subdomain order; total = offO[N].  Both buffers are allocated here.
void membership(const int64_t* offE, const int64_t* offO, const int32_t* counts, const int32_t* ext, int N,
                int64_t n, DBuf<int64_t>& memb_ptr, DBuf<int64_t>& memb, int64_t total, hipStream_t s);

// omega_flat[offO[i] + r] = Omega_i[r]; ilocal[g] = position of g in I_{part[g]}
void omega_flatten(int N, const int64_t* offE, const int64_t* offO, const int32_t* counts, const int32_t* ext,
                   int64_t total, int32_t* omega_flat, int32_t* ilocal, hipStream_t s);

// Dense Y_i = X_i^T (nt x ni, ld nt) and A_ii (ni x ni, ld ni) from CSR rows;
// buffers zero-filled by the caller.
void extract(const CsrDev& A, int N, const int64_t* offE, const int64_t* offO, const int32_t* counts,
             const int32_t* ext, double* const* Y, double* const* Aii, int64_t total_rows, hipStream_t s);

// --- vectors ---
void spmv(const CsrDev& A, const double* x, double* y, int nrhs, hipStream_t s);
void fill(double* p, int64_t n, double v, hipStream_t s);
// out[k] = sum of blocks; deterministic two-pass; out device (nrhs values)
void dot(const double* x, const double* y, int64_t n, int nrhs, double* partial, double* out, hipStream_t s);
// out[k] = x[off[k]:off[k+1]] . y[off[k]:off[k+1]] for k < nseg (off on the
// device); partial holds 512 * nseg doubles.  Deterministic order.
void dot_seg(const double* x, const double* y, const int64_t* off, int nseg, double* partial, double* out,
             hipStream_t s);
void gather(const double* x, const int32_t* idx, int64_t m, double* out, hipStream_t s);
void scatter_sum(const double* loc, const int64_t* memb_ptr, const int64_t* memb, int64_t n, double* z,
                 bool accumulate, hipStream_t s);

}  // namespace dd
