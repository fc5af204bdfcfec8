// Block-sparse (supernodal) Cholesky of the coarse operator E = Z^T A Z over
// the subdomain block graph: block (i, j) of E is nonzero only when
// subdomains i and j are neighbours in G(A).
#pragma once
#include "dense.hpp"
#include "sparse.hpp"

namespace dd {

struct UpdSrc {  // out -= A B^T with A (M x K), B (N x K), both column-major, ld = ld
    const double* A;
    const double* B;
    int ld;
    int K;
};
struct UpdJob {
    double* out;
    int ldo;
    int M, N;
    int src0, nsrc;
};
struct SolSrc {  // a (p_k x p_d) row block of panel d, ld, and the coarse offset of block d
    const double* L;
    int ld;
    int K;
    int64_t yoff;
};
struct SolNode {
    double* panel;
    int h, p;
    const double* linv;
    int64_t yoff;
    int src0, nsrc;      // forward sources (descendants)
    const int64_t* gidx; // backward: coarse index of panel rows p..h-1
    int fch0, nfch;      // forward column chunks of this node (in the level's chunk list)
    int nbch;            // backward row chunks
    int64_t part0;       // offset of this node's partial sums in the level's partial buffer
};
// A chunk of at most kSolCh consecutive columns of one forward source.
struct SolChunk {
    int node;  // index of the node within the level
    int src;   // index into the source list
    int c0, c1;
};

struct BlockChol {
    int N = 0;                               // subdomains (blocks; p = 0 blocks unused)
    std::vector<int> p;                      // block sizes
    std::vector<int64_t> yoff;               // coarse offsets (subdomain order)
    std::vector<int> pos, order;             // elimination order
    std::vector<std::vector<int>> strct;     // struct(k), sorted by pos
    std::vector<std::vector<int>> rowoff;    // row offset of each struct entry in panel k
    std::vector<int> h;                      // panel heights
    std::vector<int> lev;                    // level of each block in the elimination tree
    std::vector<std::vector<int>> by_level;
    std::vector<int64_t> poff, loff;         // panel / inverse offsets
    DBuf<double> panels, linv;
    DBuf<int64_t> gidx;                      // backward gather indices (all nodes)
    std::vector<int64_t> goff;
    // factorization update jobs per level
    std::vector<Batch<UpdJob>> upd;
    std::vector<DBuf<UpdSrc>> upd_src;
    // solve descriptors per level
    std::vector<Batch<SolNode>> sol;
    std::vector<DBuf<SolSrc>> sol_src;
    std::vector<Batch<SolChunk>> sol_ch;
    std::vector<int64_t> fwd_tiles, bwd_tiles;
    DBuf<double> tbuf, pbuf;
    int64_t nC = 0;
    double flops = 0.0;
    int64_t bytes() const { return (int64_t)(panels.bytes() + linv.bytes()); }

    // adjacency: adj[i*N + j] != 0 iff blocks i, j are coupled (symmetric)
    void symbolic(const std::vector<uint8_t>& adj, const std::vector<int>& p_, const std::vector<int64_t>& yoff_);
    void allocate(hipStream_t s);
    // pointer and ld of block (i, j), pos(i) >= pos(j), inside panel j
    double* block(int i, int j, int* ld) const;
    int factor(hipStream_t s);  // returns 0 or the first failing block + 1
    void solve(double* y, hipStream_t s);  // y := E^{-1} y (coarse vector in subdomain order)
};

}  // namespace dd
