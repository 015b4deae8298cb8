// Host-side symbolic analysis of the posterior precision (Sec. 3.2: sparse Cholesky
// with a fill-reducing node reordering, computed once per sparsity pattern and reused
// across refactorisations, Sec. 3.3).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace gmrf {

struct AnalyzeOptions {
  int32_t leaf_size = 64;       // nested-dissection leaves at or below this size stay whole
  int32_t relax_small = 8;      // always merge a child into its parent when the result has
                                // at most this many columns
  int32_t relax_mid = 32;       // ... at most this many columns and <= 50% explicit zeros
  double relax_frac_mid = 0.5;
  int32_t relax_big = 128;      // ... at most this many columns and <= 15% explicit zeros
  double relax_frac_big = 0.15;
  double relax_frac_any = 0.03; // any size with <= 3% explicit zeros
  int32_t nb = 64;              // dense block width of the front kernels
};

// Everything the numeric phase needs, in pivot (permuted, postordered) numbering.
struct Symbolic {
  int64_t n = 0;
  std::vector<int32_t> perm;      // perm[k] = original index of pivot k
  std::vector<int32_t> iperm;     // iperm[perm[k]] = k
  std::vector<int32_t> parent;    // column elimination tree
  std::vector<int64_t> colcount;  // exact column counts of L, diagonal included

  // supernodes: contiguous pivot ranges [sfirst[s], sfirst[s+1])
  int32_t ns = 0;
  std::vector<int32_t> sfirst;    // ns+1
  std::vector<int32_t> sparent;   // ns, -1 for roots
  std::vector<int64_t> rowptr;    // ns+1, offsets into rows
  std::vector<int32_t> rows;      // front index list F_s (sorted pivots); first p_s = columns
  std::vector<int32_t> relpos;    // aligned with rows; for the R part (index >= p_s) the
                                  // position of that pivot in the parent's front, else -1
  std::vector<int32_t> depth;     // roots have depth 0
  std::vector<int32_t> child_ptr; // ns+1, CSR of children (ascending)
  std::vector<int32_t> child_idx;
  int32_t max_depth = -1;

  // storage plan
  std::vector<int64_t> Loff;      // panel n_s x p_s (column-major, ld n_s) in L storage
  int64_t Lsize = 0;
  std::vector<int64_t> Woff;      // square n_s x n_s front inside its depth's buffer
  int64_t Wsize[2] = {0, 0};      // buffer for even / odd depths
  std::vector<int64_t> Doff;      // nb x nb inverse diagonal blocks, ceil(p/nb) per supernode
  int64_t Dsize = 0;
  std::vector<int64_t> Voff;      // front vectors (length n_s) inside a depth's vector buffer
  int64_t Vsize[2] = {0, 0};

  // counts (exact pattern of L, relaxation zeros excluded)
  int64_t nnzL = 0;
  double flops_factor = 0.0;      // sum c_j^2
  double flops_selinv = 0.0;      // 2 sum c_j^2
  double flops_solve = 0.0;       // 4 nnz(L) - 2n per right-hand side
  int64_t stored_L = 0;           // sum n_s p_s - p_s(p_s-1)/2 (supernodal storage incl. zeros)

  int32_t p(int32_t s) const { return sfirst[s + 1] - sfirst[s]; }
  int32_t nf(int32_t s) const { return (int32_t)(rowptr[s + 1] - rowptr[s]); }
};

// pattern: CSR (both triangles, sorted, symmetric, diagonal present) of the n x n matrix.
// coords: optional n x dim node coordinates (row-major) steering the dissection.
// perm_in: optional fill-reducing order (perm_in[k] = original index of pivot k) used
// instead of the nested dissection (then postordered like it).
// Returns an empty string on success, else an error message.
std::string analyze(int64_t n, const int64_t* rp, const int32_t* ci, const double* coords,
                    int dim, const AnalyzeOptions& opt, Symbolic& out, const int32_t* perm_in = nullptr);

// Fill-reducing nested-dissection ordering only (exposed for host tests).
void nested_dissection(int64_t n, const int64_t* rp, const int32_t* ci, const double* coords,
                       int dim, int32_t leaf, std::vector<int32_t>& perm);

// Exact column counts of L for a given pivot order (elimination-tree row subtrees).
void column_counts(int64_t n, const int64_t* rp, const int32_t* ci,
                   const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
                   const std::vector<int32_t>& parent, std::vector<int64_t>& cc);

void elimination_tree(int64_t n, const int64_t* rp, const int32_t* ci,
                      const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
                      std::vector<int32_t>& parent);

}  // namespace gmrf
