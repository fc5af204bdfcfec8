// Graph, index-map, extraction and vector kernels (integer parts bit-exact).
#pragma once
#include "common.hpp"

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

// --- overlap layers: dist[i*n + v] in {0..delta+1, 255} ---
void layers(const CsrDev& A, const int32_t* part, int N, int delta, uint8_t* dist, hipStream_t s);
// counts[3*i + {0,1,2}] = |I_i|, |Gamma_i|, |Delta_i|
void layer_counts(const uint8_t* dist, int64_t n, int N, int delta, int32_t* counts, hipStream_t s);
// ext[offE[i] + ...] = [I_i, Gamma_i, Delta_i] each ascending
void layer_compact(const uint8_t* dist, int64_t n, int N, int delta, const int64_t* offE, const int32_t* counts,
                   int32_t* ext, hipStream_t s);

// Exclusive prefix sum of int32 counts into int64 offsets (n+1 entries), one workgroup.
void scan_counts(const int32_t* counts, int64_t n, int64_t* offsets, hipStream_t s);

// Membership of every node: memb_ptr[g]..memb_ptr[g+1] lists positions (in the
// concatenated Omega buffer, offO[i] + local index) of the subdomains containing g,
// in subdomain order.
void membership_counts(const uint8_t* dist, int64_t n, int N, int delta, int32_t* cnt, hipStream_t s);
void membership_fill(const uint8_t* dist, int64_t n, int N, int delta, const int64_t* offE, const int64_t* offO,
                     const int32_t* counts, const int32_t* ext, const int64_t* memb_ptr, int64_t* memb,
                     hipStream_t s);

// omega_flat[offO[i] + r] = Omega_i[r]; ilocal[g] = position of g in I_{part[g]}
void omega_flatten(int N, const int64_t* offE, const int64_t* offO, const int32_t* counts, const int32_t* ext,
                   int64_t total, int32_t* omega_flat, int32_t* ilocal, hipStream_t s);

// Dense Y_i = X_i^T (nt x ni, ld nt) and A_ii (ni x ni, ld ni) from CSR rows;
// buffers zero-filled by the caller.
void extract(const CsrDev& A, int N, int delta, int64_t n, const uint8_t* dist, const int64_t* offE,
             const int64_t* offO, const int32_t* counts, const int32_t* ext, double* const* Y, double* const* Aii,
             int64_t total_rows, hipStream_t s);

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
