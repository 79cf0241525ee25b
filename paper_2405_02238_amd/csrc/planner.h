// HEGMM-En planner (Algorithm 2 of the paper, Section III-C).
//
// Given (m, l, n) and the slot count S of one rotation row, decides the
// orientation (duplicate A, or transpose so that B is duplicated), the
// duplication count d (Theorems 5/6), the packed layout (column-major with
// column stride M = d * m_o), the loop trip count K = min(m_o, l), the
// diagonals of every eps^k / omega^k transform with their slot masks, the
// fold that gathers the d row blocks, and the inner-dimension blocking used
// when the packed operands do not fit S slots.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace hg {

struct Term {
    int z;      // left-rotation amount (unreduced; may be negative)
    int mask;   // index into Plan::masks, or -1: no mask multiply
};

struct Plan {
    int m = 0, l = 0, n = 0;
    bool transposed = false;
    int mo = 0, no = 0;   // oriented problem: X (mo x l) times Y (l x no)
    int nb = 1, lb = 0;   // inner blocks and block length (zero padded)
    int d = 1, M = 0, K = 0, W = 0;
    std::vector<std::vector<Term>> eps, omega;  // per k
    std::vector<int> fold;                      // h * mo, h = 0..d-1
    std::vector<std::vector<uint8_t>> masks;    // S bytes each, 1 = slot kept
    int method = 2;                             // 2: HEGMM-En (Algorithm 2); 1: HEGMM (Algorithm 1);
                                                // 3: Algorithm 1 with sigma / tau in the cloud
    std::vector<Term> sigma, tau;               // method 3: the transforms applied to X and Y first
    std::vector<int> rotations(int S) const;    // distinct nonzero z mod S
    int key_switched_terms(int S) const;        // terms that need a key switch
};

// Throws std::invalid_argument when a dimension is not positive and
// std::range_error when the shape cannot be planned into S slots.
// min_blocks > 1 splits the inner dimension into at least that many blocks
// (capped at l) even when fewer would fit (method 2 only).
// method 2: HEGMM-En; method 1: the paper's Algorithm 1 (HEGMM), sigma and
// tau applied by the client, column-major or (when that needs fewer
// key-switched diagonals) row-major flattening, no duplication, no blocking;
// method 3: Algorithm 1 with the operands packed as they are and sigma / tau
// applied to the ciphertexts (2 min(mo, l) - 1 and 2 min(no, l) - 1
// diagonals, Theorems 1 and 2).
Plan make_plan(int m, int l, int n, int S, int method = 2, int min_blocks = 1);

// Client packing: the slot vector (length S, values in [0, t)) of the left
// (side 0) or right (side 1) operand of the oriented problem for inner block
// `block`.  X is the caller's matrix that feeds that side, row-major: side 0
// takes A (m x l), or B (l x n) when the plan is transposed; side 1 takes B,
// or A when transposed.
std::vector<uint64_t> pack_operand(const Plan &p, int side, const int64_t *X, int block, uint64_t t, int S);

// The packed side fed by the caller's matrix `role` (0 = A, 1 = B).
inline int side_of_role(const Plan &p, int role) { return p.transposed ? 1 - role : role; }

// Position of result entry C[i][j] in the result's slot vector.
inline int result_slot(const Plan &p, int i, int j) {
    return p.transposed ? (j + i * p.M) : (i + j * p.M);
}

}  // namespace hg
