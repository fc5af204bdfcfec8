// Local solves of the additive apply (2.1) for several right-hand sides at
// once: every W_i = L_i^{-1} is read once per group of up to kMrhs columns.
#pragma once
#include "dense.hpp"

namespace dd {

constexpr int kMrhs = 8;  // right-hand sides per pass

// As TrmvItemT, with column k of x, y and part at x + k xs, y + k ys, part + k ps.
template <class TW>
struct TrmvMItem {
    const TW* W;
    int ld;
    int n;
    double* x;
    double* y;
    double* part;
    int64_t xs, ys, ps;
};

// x_k := W^T W x_k for k < nrhs (nrhs <= kMrhs); every column's sums run in
// the order of trinv_apply_vb, so each column equals its single-column result
void trinv_apply_multi_vb(Batch<TrmvMItem<double>>& t, int nrhs, hipStream_t s);
void trinv_apply_multi_vb(Batch<TrmvMItem<float>>& t, int nrhs, hipStream_t s);

}  // namespace dd
