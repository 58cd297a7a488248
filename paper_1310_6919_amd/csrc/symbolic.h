// Host symbolic phase: everything about structure, computed once per problem.
//
// Section 2.1: aggregate pattern -> ordering -> chordal extension (the fill
// of Y = N N^T) -> cliques.  Section 3.1: supernodes of the symbolic
// factorisation serve as the cliques C_r (row sets) and S_r (column sets);
// Lhat and N share one storage structure.
//
// Two partitions of the columns are kept:
//   cliques  the fundamental supernodes.  Algorithm 1 and the clique-wise
//            step length run on these (exact E).
//   blocks   storage panels: consecutive supernodes along an elimination-tree
//            chain, or consecutive sibling subtrees whose rows below the block
//            do not grow, merged up to a width limit (explicit zeros allowed),
//            or a wide supernode cut into pieces.  Every column's exact structure
//            lies inside its block's row list, so factors stored this way are
//            the same matrices; the zeros only pad the dense panel work.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace sdpc {

struct Symbolic {
    int n = 0;
    std::vector<int> perm;            // perm[pos] = original index
    std::vector<int> pos;             // pos[orig] = position
    // exact chordal structure (positions)
    std::vector<int> parent;          // elimination tree, -1 for roots
    std::vector<int64_t> sptr;        // struct(j) = sidx[sptr[j]..sptr[j+1]), sorted, starts with j
    std::vector<int> sidx;
    // cliques (fundamental supernodes)
    int ncl = 0;
    std::vector<int> cl_first;        // ncl + 1
    // storage blocks
    int nb = 0;
    std::vector<int> bl_first;        // nb + 1 column ranges
    std::vector<int64_t> bl_rptr;     // rows of block b: bl_rows[bl_rptr[b]..bl_rptr[b+1])
    std::vector<int> bl_rows;         // own columns first (ascending), then the rest ascending
    std::vector<int64_t> bl_off;      // panel offsets, nb + 1; panel b is h_b x w_b column-major
    std::vector<int> bl_parent;       // block of parent(last column), -1 at a root
    std::vector<int> bl_subfirst;     // smallest column in the block's elimination subtree
    std::vector<int> col_block;       // block of every column
    int64_t nslot = 0;
    std::vector<uint8_t> isE;         // slot lies in the exact E (lower triangle)
    int max_h = 0, max_w = 0, max_clique = 0;

    // slot of (i, j), i >= j positions, -1 if (i, j) is not stored
    int64_t slot(int i, int j) const;
};

struct SymbolicOptions {
    int ordering = 0;                 // 0 natural, 1 minimum degree, 2 user
    const int32_t *user_perm = nullptr;
    int block_width = 32;
    int max_block_entries = 8192;     // h * w limit of one panel (doubles)
    int merge_siblings = 1;           // also merge consecutive sibling subtrees whose tail rows do not grow
};

// Builds everything from the lower-triangle aggregate pattern (original
// indices, row >= col, diagonal included).  Returns "" on success, else a
// message.
std::string build_symbolic(int n, const std::vector<int> &arow, const std::vector<int> &acol,
                           const SymbolicOptions &opt, Symbolic &S);

// Exact minimum-degree order (elimination game, lowest index on ties).
std::vector<int> min_degree_order(int n, const std::vector<int> &arow,
                                  const std::vector<int> &acol);

// Register-allocation style slot assignment for the solves: for the forward
// sweep (blocks ascending) a row is live from the first block whose update
// reaches it until its own block; for the backward sweep (blocks descending)
// from its own block until the last block that reads it.  Intervals are
// coloured greedily; returns the number of slots used.
// With delay set, a slot freed at a block becomes free for rows of the next block on,
// so no block step reads a slot as one of its own rows while writing it as a row below
// (or the reverse on the backward walk); without it, a block's own rows give their
// slots to the rows it brings to life, which needs fewer slots.
struct SolveSlots {
    int nfwd = 0, nbwd = 0;
    std::vector<int> fwd;             // per row: forward slot, -1 if never updated
    std::vector<int> bwd;             // per row: backward slot, -1 if never read
    std::vector<int> birth;           // per row: first block that updates it, -1 if none
};
SolveSlots build_solve_slots(const Symbolic &S, bool delay);

}  // namespace sdpc
