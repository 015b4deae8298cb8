// Device-side data of the numeric phase and the launch wrappers of the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gmrf {

constexpr int kTile = 64;     // dense tile edge (rows/cols) of the front kernels
constexpr int kNB = 64;       // diagonal block width; equals the analysis option nb
constexpr int kNB2 = 256;     // outer block width of the two-level blocking
constexpr int kBigTile = 128; // tile edge of the long-K MFMA kernels
constexpr int kExtCols = 4;   // columns per work-group of the extend-add and the Sigma gather

// Read-only symbolic arrays on the device (pivot numbering).
struct DevSym {
  int64_t n;
  const int32_t* perm;      // pivot -> original
  const int32_t* sfirst;    // ns+1
  const int64_t* rowptr;    // ns+1
  const int32_t* rows;      // front index lists
  const int32_t* relpos;    // child R -> parent front position
  const int32_t* child_ptr; // ns+1
  const int32_t* child_idx;
  const int64_t* Loff;
  const int64_t* Woff;
  const int64_t* Doff;
  const int64_t* Voff;
};

// One batched launch over a list of fronts; prefix[i] = first work-group of front i.
struct LaunchList {
  const int32_t* fronts;
  const int64_t* prefix;
  const int2* wgmap;        // per work-group (list index, local index), or null
  const int32_t* aux;       // two ints per listed front (meaning set by the kernel), or null
  int32_t count;
  int64_t total;            // number of work-groups
};

template <typename T>
struct NumBufs {
  T* L;            // supernodal panels
  T* D;            // inverse diagonal blocks (nb x nb each)
  double* piv;     // FP64 pivots L_jj (pivot order)
  T* Wcur;         // front buffer of the current depth
  T* Wchild;       // front buffer of the child depth
  int32_t* status; // first failing pivot (INT32_MAX if none)
};

// ---- assembly (original numbering) ----
void launch_assemble_qpost(hipStream_t st, int64_t nnzq, const double* qval,
                           const int64_t* cptr, const int32_t* cpair, const int32_t* arow,
                           const double* aval, const double* qeps, double* qpost);
void launch_obs_residual(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci,
                         const double* aval, const double* qeps, const double* y,
                         const double* b, const double* mu, double* rvec);
void launch_at_times(hipStream_t st, int64_t n, const int64_t* atp, const int32_t* ati,
                     const int32_t* arow, const double* aval, const double* rvec, double* h);
void launch_equilibrate(hipStream_t st, int64_t n, int64_t nnzq, const int64_t* qdiag,
                        const int32_t* qrow, const int32_t* qcol, const double* qpost,
                        int32_t* sexp, double* scale, double* qhat);
// dQ_post = dq + da^T Q_eps A + A^T Q_eps da + A^T diag(dqeps) A on Q's pattern (da, dqeps nullable)
void launch_assemble_dqpost(hipStream_t st, int64_t nnzq, const double* dq, const int64_t* cptr,
                            const int32_t* cpair, const int32_t* arow, const double* aval, const double* da,
                            const double* qeps, const double* dqeps, double* out);
// y = V x on A's pattern (values V, m rows)
void launch_spmv_obs(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* v,
                     const double* x, double* y);
// r = y - b - V x on A's pattern (b nullable)
void launch_obs_resid_plain(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* v,
                            const double* y, const double* b, const double* x, double* r);
// conjugate gradients with device scalars sc = (r^T z, p^T q, new r^T z): x += alpha p,
// r -= alpha q (alpha = sc0 / sc1); p = z + beta p (beta = sc2 / sc0), then sc0 = sc2
void launch_cg_xr(hipStream_t st, int64_t n, const double* sc, const double* p, const double* q, double* x,
                  double* r);
void launch_cg_p(hipStream_t st, int64_t n, double* sc, const double* z, double* p);
void launch_copy_f64(hipStream_t st, int64_t n, const double* a, double* b);
// z = r / diag(Q) (qdiag: index of each row's diagonal entry)
void launch_jacobi(hipStream_t st, int64_t n, const int64_t* qdiag, const double* qv, const double* r, double* z);
constexpr int kSelChunk = 512;   // rows of R' per split-K partial of the Sigma diagonal blocks
constexpr int kCgPartials = 3 * 2048;  // partial sums of launch_cg_iteration
// one Jacobi-preconditioned CG iteration: q = Q p with the partials of p^T q (summed into
// sc[2]); x, r, z updates with the partials of r^T z (summed into sc[1 - cur]) and r^T r;
// p update.  sc[cur] holds r^T z on entry.  sc needs 6 doubles; part: kCgPartials doubles.
void launch_cg_iteration(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                         const int64_t* qdiag, double* sc, int cur, double* x, double* r, double* z, double* p,
                         double* q, double* part);
// out[0] = ||r|| from the r^T r partials of the last launch_cg_iteration (out[2] is used
// for the squared norm)
void launch_partial_norm(hipStream_t st, const double* part, double* out);
// Rao-Blackwellised marginal variances from k draws of N(0, Q^-1)
void launch_rbmc(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* qv,
                 const int64_t* qdiag, int64_t k, const double* xs, double* var);
// mode 0: a * b, 1: a / b, 2: log(a), 3: sqrt(a) * b, elementwise
void launch_elementwise(hipStream_t st, int64_t n, int mode, const double* a, const double* b, double* out);
void launch_fill_i32(hipStream_t st, int32_t* p, int64_t n, int32_t v);
void launch_fill_f64(hipStream_t st, double* p, int64_t n, double v);

// ---- factorisation ----
// lower triangles (diagonal included) of the listed fronts, 4 columns per work-group
template <typename T> void launch_zero_lower(hipStream_t st, const DevSym& S, const LaunchList& L, T* W);
template <typename T> void launch_scatter(hipStream_t st, int64_t cnt, const int64_t* map_e,
                                          const int64_t* map_off, const double* qhat, T* W);
template <typename T> void launch_extend_add(hipStream_t st, const DevSym& S, const LaunchList& L,
                                             int slot, const T* Wchild, T* Wcur);
template <typename T> void launch_potrf(hipStream_t st, const DevSym& S, const LaunchList& L,
                                        int step, NumBufs<T> B);
template <typename T> void launch_trsm(hipStream_t st, const DevSym& S, const LaunchList& L,
                                       int step, NumBufs<T> B);
// mode 0: inner panel update after 64-block `step`; 1: outer update after the last
// 64-block of a 256-wide outer block; 2: trailing SYRK of the update matrix
template <typename T> void launch_update(hipStream_t st, const DevSym& S, const LaunchList& L,
                                         int step, int mode, NumBufs<T> B);
template <typename T> void launch_copy_L(hipStream_t st, const DevSym& S, const LaunchList& L,
                                         NumBufs<T> B);
// partial sums per block of the log-determinant reduction
constexpr int kLdParts = 64;
// part: nblocks * kLdParts doubles of scratch, each written before it is read
void launch_logdet(hipStream_t st, int64_t nblocks, const int64_t* bptr, const int32_t* bpiv,
                   const int32_t* perm, const double* piv, const int32_t* sexp, double* part, double* out);

// ---- triangular solves (front vectors in FP64, L in T) ----
struct SolveBufs {
  double* xp;      // n x nrhs, pivot order, ld n
  double* Vcur;    // front vectors of the current depth
  double* Vchild;  // front vectors of the adjacent depth
  int nrhs;
};
template <typename T> void launch_fvec_init(hipStream_t st, const DevSym& S, const LaunchList& L, SolveBufs V);
template <typename T> void launch_fvec_extend(hipStream_t st, const DevSym& S, const LaunchList& L, int slot, SolveBufs V);
// solves blocked by 256-wide outer blocks (forward left to right, backward from the right)
template <typename T> void launch_fwd_block(hipStream_t st, const DevSym& S, const LaunchList& L, int t,
                                            const T* D2, const int64_t* D2off, SolveBufs V);
// inverses of the 256-wide diagonal blocks (Lbase: front buffer if from_front, else L storage)
template <typename T> void launch_inv256(hipStream_t st, const DevSym& S, const LaunchList& L, const T* Lbase,
                                         int from_front, const T* Dinv, const int64_t* D2off, T* D2, T* D2T);
template <typename T> void launch_fwd_outer(hipStream_t st, const DevSym& S, const LaunchList& L, int t,
                                            const T* Lp, SolveBufs V);
template <typename T> void launch_bwd_part(hipStream_t st, const DevSym& S, const LaunchList& L, int t,
                                           const T* Lp, SolveBufs V, double* part);
template <typename T> void launch_bwd_block(hipStream_t st, const DevSym& S, const LaunchList& L,
                                            const LaunchList& Lpart, int t, const T* D2T, const int64_t* D2off,
                                            SolveBufs V, const double* part);
// Solves with one right-hand side: one work-group per 64-row chunk task (front, chunk) in
// dependency order; ticket: the launch's counter (zero before the launch), prog:
// per-supernode count of published x blocks (zero before the pass), err: set if a
// dependency wait exceeded its spin limit.
struct FusedTasks {
  const int2* task;
  int32_t* ticket;
  int32_t* prog;
  int32_t* err;
  int64_t count;             // work-groups of the launch = task groups
  const int32_t* group;      // group g holds tasks group[g] .. group[g + 1] - 1, in order
};
// Whole-forest solves (one launch per pass over every depth): the front vectors' update
// parts live in one array (uoff per front), a front's rows gather their children's update
// entries through a row-CSR map (gptr over rows of all fronts, roff per front; gsrc =
// positions in the update array, children in fixed order), and kids[s] counts the
// children's chunks whose update rows are final (need[s] of them).
struct ForestBufs {
  const int32_t* parent;   // supernodal parent, -1 for roots
  const int32_t* need;     // per front: number of child chunks holding update rows
  int32_t* kids;           // per front: child chunks finished (zero before the pass)
  const int64_t* roff;     // per front: first row entry in gptr
  const int64_t* gptr;     // row-CSR into gsrc
  const int64_t* gsrc;     // update-array positions of the children's entries
  const int64_t* uoff;     // per front: offset of its update part in U
  double* U;               // update parts of all fronts
};
// one launch over the whole forest (tasks deepest first for the forward, from the roots
// for the backward); xp holds the right-hand side on entry and the solution on exit.
// skip (device, nullable): when skip[0] == 0 the launch does nothing, which leaves a zero
// right-hand side as its own solution (the gated refinement passes).
template <typename T> void launch_fwd_forest(hipStream_t st, const DevSym& S, FusedTasks F, ForestBufs G,
                                             const T* Lp, const T* D, double* xp, const double* skip = nullptr);
// nrhs right-hand sides (column r at xp + r * ldx) in one backward pass
template <typename T> void launch_bwd_forest(hipStream_t st, const DevSym& S, FusedTasks F, ForestBufs G,
                                             const T* Lp, const T* D, double* xp, int nrhs = 1, int64_t ldx = 0,
                                             const double* skip = nullptr);
// xp = gate[0] * S P src (gate nullable = 1)
void launch_permute_in(hipStream_t st, int64_t n, int nrhs, const int32_t* perm, const double* scale,
                       const double* src, int64_t lds, double* xp, const double* gate = nullptr);
// refinement gate: norms = (||h||, ||r||); gate[0] = 1 while ||r|| > tol ||h||, gate[1]
// counts the corrections; record != 0 writes (||r||/||h||, gate[1]) to rec[0..1]
void launch_refine_gate(hipStream_t st, const double* norms, double tol, double* gate, double* rec, int record);
void launch_permute_in_f32(hipStream_t st, int64_t n, int nrhs, const float* z, double* xp);
void launch_permute_out(hipStream_t st, int64_t n, int nrhs, const int32_t* perm, const double* scale,
                        const double* xp, const double* add, int64_t ldadd, double* out, int64_t ldo,
                        int accumulate);
void launch_resid(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                  const double* h, const double* x, double* r);
void launch_matern_values(hipStream_t st, int64_t nnz, const double* mv, const double* sv, const double* smsv,
                          double kappa, double tau, double* q, double* dq);
void launch_spmv(hipStream_t st, int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                 const double* x, double* y);
void launch_weighted_resid(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* aval,
                           const double* qeps, const double* y, const double* b, const double* x, double* w);
// Gauss-Newton (Burgers): linearisation, batched line search (part: 10 * 256 doubles;
// quad: u^T Q u, u^T Q d, d^T Q d), direction and update
void launch_burgers_linearize(hipStream_t st, int64_t nx, int64_t nt, double dt, double nu, const double* mass,
                              const double* s3, const double* u, const int64_t* arp, double* aval, double* b);
void launch_gn_linesearch(hipStream_t st, int64_t nx, int64_t nt, double dt, double nu, const double* mass,
                          const double* s3, const double* u, const double* d, const double* y, const double* qeps,
                          const int64_t* arp, const int32_t* aci, const double* aval, double* part,
                          const double* quad, double* sel, double* rec);
// Gauss-Newton with a pointwise power nonlinearity: f_r(u) = (lin u)_r + nl_coef[r] u[nl_col[r]]^power
void launch_pw_linearize(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* lin,
                         const int32_t* nl_col, const double* nl_coef, int power, const double* u, double* aval,
                         double* b);
void launch_pw_linesearch(hipStream_t st, int64_t m, const int64_t* arp, const int32_t* aci, const double* lin,
                          const int32_t* nl_col, const double* nl_coef, int power, const double* u, const double* d,
                          const double* y, const double* qeps, const double* aval, double* part, const double* quad,
                          double* sel, double* rec);
void launch_gn_direction(hipStream_t st, int64_t n, const double* x, const double* u, double* d);
void launch_gn_update(hipStream_t st, int64_t n, const double* sel, const double* d, double* u);
void launch_add(hipStream_t st, int64_t n, const double* a, const double* b, double* out);
void launch_norm2(hipStream_t st, int64_t n, const double* v, double* partial, double* out);

// ---- selected inversion ----
template <typename T>
struct SelBufs {
  const T* L;
  const T* D;
  T* Scur;         // square Sigma fronts of the current depth
  T* Spar;         // square Sigma fronts of the parent depth
  T* Y;            // 256 x n_s scratch per front (offset Voff * 256), block columns contiguous
  T* part;         // split-K partials of the diagonal Sigma blocks
  T* gpart;        // split-K partials of Sigma[R', K] (128 x 128 per work-group)
};
template <typename T> void launch_sel_gather(hipStream_t st, const DevSym& S, const LaunchList& L, const int32_t* sparent, SelBufs<T> B);
// two-level selected inversion (256-wide outer blocks counted from the right by `step`)
template <typename T> void launch_sel_Y2(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                         SelBufs<T> B, const int64_t* D2off, const T* D2);
template <typename T> void launch_sel_gemm2(hipStream_t st, const DevSym& S, const LaunchList& L, int step, SelBufs<T> B);
template <typename T> void launch_sel_gemm_reduce(hipStream_t st, const DevSym& S, const LaunchList& L, int step,
                                                  SelBufs<T> B);
// FP32 Sigma[R', K] in 256 x 256 tiles (one work-group per 256 rows and K part, split over K
// like launch_sel_gemm2; partials 256 x 256)
void launch_sel_gemm4(hipStream_t st, const DevSym& S, const LaunchList& L, int step, SelBufs<float> B);
// FP32 trailing SYRK of the update matrices in 256 x 256 tiles
void launch_syrk4(hipStream_t st, const DevSym& S, const LaunchList& L, NumBufs<float> B);
// FP32 left-looking update of outer block K of the pivot panels from all earlier outer
// blocks in 256 x 256 tiles (split-K partials in part, summed by launch_panel_red4)
void launch_panel_upd4(hipStream_t st, const DevSym& S, const LaunchList& L, int K, NumBufs<float> B, float* part);
void launch_panel_red4(hipStream_t st, const DevSym& S, const LaunchList& L, int K, NumBufs<float> B,
                       const float* part);
template <typename T> void launch_sel_part2(hipStream_t st, const DevSym& S, const LaunchList& L, int step, SelBufs<T> B);
template <typename T> void launch_sel_fin2(hipStream_t st, const DevSym& S, const LaunchList& L, const LaunchList& Lpart,
                                           int step, SelBufs<T> B, const int64_t* D2off, const T* D2);
template <typename T> void launch_sel_extract(hipStream_t st, const DevSym& S, const LaunchList& L, SelBufs<T> B,
                                              const double* scale, double* var);
template <typename T> void launch_sel_pattern(hipStream_t st, int64_t cnt, const int64_t* map_e,
                                              const int64_t* map_off, const int32_t* qrow,
                                              const int32_t* qcol, const double* scale,
                                              const T* Scur, double* sigq);
void launch_dot(hipStream_t st, int64_t n, const double* a, const double* b, double* partial, double* out);

}  // namespace gmrf
