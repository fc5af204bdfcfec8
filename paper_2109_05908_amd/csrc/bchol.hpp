// Block-sparse supernodal Cholesky of the coarse operator E = Z^T A Z over
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
    int lower;  // diagonal block (A == B in every source): lower tiles only
};
// Forward-solve source: rows of a descendant supernode's panel that belong to
// the target supernode (a contiguous row range of the panel), and where each
// of those rows lands within the target.
struct SolSrc {
    const double* L;     // first of the rows inside the source panel
    int ld;              // source panel height
    int K;               // source supernode width (columns)
    int rows;            // number of rows
    int64_t xoff;        // permuted coarse offset of the source supernode
    const int32_t* ridx; // row -> row within the target supernode
};
struct SolNode {
    double* panel;
    int h, w;            // panel height and width (supernode width)
    int64_t start;       // permuted coarse offset of the supernode
    const int64_t* gidx; // backward: permuted coarse index of panel rows w..h-1
    int fch0, nfch;      // forward column chunks of this node (in the level's chunk list)
    int nbch;            // backward row chunks
    int64_t part0;       // offset of this node's partial sums in the level's partial buffer
};
// A chunk of at most kSolCh consecutive columns of one forward source.
struct SolChunk {
    int node;  // index of the node within the level
    int src;   // index into the level's source list
    int c0, c1;
};

struct BlockChol {
    // blocks (subdomains; p = 0 blocks unused), in subdomain order
    int N = 0;
    std::vector<int> p;                      // block sizes
    std::vector<int64_t> yoff;               // coarse offsets (subdomain order)
    std::vector<int> pos, order;             // block elimination order (weighted minimum degree)
    std::vector<std::vector<int>> bstruct;   // struct of each block, sorted by pos
    // supernodes: runs of consecutive blocks in elimination order along a chain
    // of the elimination tree, each block's struct = the next block U its struct
    int NS = 0;
    std::vector<int> sn, cof;                // block -> supernode, column offset inside it
    std::vector<std::vector<int>> members;   // supernode -> blocks in elimination order
    std::vector<int> w, h;                   // supernode width and panel height
    std::vector<std::vector<int>> srows;     // supernode -> struct blocks (rows below the diagonal part)
    std::vector<std::vector<int>> srowoff;   // panel row offset of each struct block
    std::vector<int64_t> start, bstart;      // permuted coarse offsets of supernodes and blocks
    std::vector<int> lev;
    std::vector<std::vector<int>> by_level;  // supernodes per elimination-tree level
    std::vector<int64_t> poff, loff, goff;
    DBuf<double> panels, linv;
    DBuf<int64_t> gidx, perm;                // perm: subdomain-order coarse index -> permuted index
    DBuf<int32_t> ridx;
    // factorization update jobs per level
    std::vector<Batch<UpdJob>> upd;
    std::vector<DBuf<UpdSrc>> upd_src;
    // solve descriptors per level
    std::vector<Batch<SolNode>> sol;
    std::vector<DBuf<SolSrc>> sol_src;
    std::vector<Batch<SolChunk>> sol_ch;
    std::vector<Batch<TrmvItem>> sol_trf, sol_trb;  // diagonal steps with the explicit inverses
    std::vector<int64_t> fwd_tiles, bwd_tiles, part_len;
    DBuf<double> tbuf, pbuf, ybuf, trpart;
    int64_t nC = 0;
    double flops = 0.0;
    int64_t bytes() const { return (int64_t)(panels.bytes() + linv.bytes()); }

    // adjacency: adj[i*N + j] != 0 iff blocks i, j are coupled (symmetric)
    void symbolic(const std::vector<uint8_t>& adj, const std::vector<int>& p_, const std::vector<int64_t>& yoff_);
    void allocate(hipStream_t s);
    // pointer and ld of block (i, j), pos(i) >= pos(j), inside the panel of j's
    // supernode; nullptr if (i, j) is outside the factor's structure
    double* block(int i, int j, int* ld) const;
    int factor(hipStream_t s);  // returns 0 or the first failing block + 1
    void solve(double* y, hipStream_t s);  // y := E^{-1} y (coarse vector in subdomain order)
};

}  // namespace dd
