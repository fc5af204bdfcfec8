// Coarse space: Z (2.1, 3.3) and E = Z^T A Z, restriction / prolongation.
#pragma once
#include "dense.hpp"
#include "sparse.hpp"

namespace dd {

// Everything the coarse kernels need to know about one level's subdomains.
struct SubInfo {
    int N;
    const int32_t* counts;    // 3N: nI, nG, nD
    const int64_t* offE;      // N+1
    const int64_t* offO;      // N+1
    const int32_t* ext;       // concatenated Omega~_i
    const int32_t* part;      // n
    const int32_t* ilocal;    // n: position of g inside I_{part[g]}
    const int32_t* pcnt;      // N: kept modes p_i
    const int64_t* offC;      // N+1: coarse offsets
    double* const* Z;         // Z_i (nI x p_i, ld nI)
};

// pair counts cnt[j*N + i] = #rows of Omega_j owned by subdomain i
void pair_counts(const SubInfo& S, int32_t* cnt, hipStream_t s);
// fill per-pair row lists: zr (row in Z_i), pr (row in P_j)
void pair_fill(const SubInfo& S, const int64_t* pairoff, int32_t* cursor, int32_t* zr, int32_t* pr, hipStream_t s);
// P_j = A(Omega_j, Omega_Ij) Z_j   (n_j x p_j, ld n_j)
void build_p(const CsrDev& A, const SubInfo& S, double* const* P, const std::vector<int>& hni,
             const std::vector<int>& hp, hipStream_t s);

struct PairItem {
    int i, j;
    int nrows;
    int64_t rows;  // offset into zr / pr
    double* out;   // destination of block (i, j): p_i x p_j, leading dimension ldo
    int64_t ldo;
};
// out_q(a, b) = sum_k Z_i(zr_k, a) P_j(pr_k, b) for every pair q = (i, j)
void assemble_e(const SubInfo& S, const PairItem* dpairs, const std::vector<PairItem>& hpairs,
                const std::vector<int>& hp, double* const* P, const int32_t* zr, const int32_t* pr, hipStream_t s);

// adj[i*N + j] = 1 when an edge of G(A) joins Omega_Ii and Omega_Ij (i != j)
void block_adjacency(const CsrDev& A, const int32_t* part, int N, uint8_t* adj, hipStream_t s);

// y[offC_i + a] = sum_r Z_i(r, a) x[I_i(r)]
void restrict_coarse(const SubInfo& S, int64_t nC, const double* x, double* y, hipStream_t s);
// z[I_i(r)] += sum_a Z_i(r, a) y[offC_i + a]
void prolong_coarse(const SubInfo& S, const int64_t* offI, int64_t nI_total, const double* y, double* z, hipStream_t s);

}  // namespace dd
