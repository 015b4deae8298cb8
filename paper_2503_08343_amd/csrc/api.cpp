// C ABI of libgmrf.so: pattern intake and validation, assembly maps, the device
// execution plan derived from the symbolic analysis, and the drivers of the numeric
// phases (factor, solves with iterative refinement, sampling, selected inversion).
#include "gmrf.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "kernels.h"
#include "symbolic.h"

using namespace gmrf;

// Workspace of gmrf_logdet_noalloc: the per-block partial sums of the log-determinant
// (kLdParts per block) in a fixed device array, so that the call allocates nothing.
// Each device holds its own copy for the life of the process (4 MiB); its device
// address is looked up once per device (gmrf_create) and only that address is handed
// to kernels.
constexpr int64_t kNoAllocMaxBlocks = 8192;

static __device__ __align__(256) double scratch[kNoAllocMaxBlocks * kLdParts];

namespace {

template <typename T>
struct DevArr {
  T* p = nullptr;
  size_t n = 0;
  DevArr() = default;
  DevArr(const DevArr&) = delete;
  DevArr& operator=(const DevArr&) = delete;
  ~DevArr() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t alloc(size_t cnt) {
    if (cnt <= n && p) return hipSuccess;
    release();
    size_t bytes = std::max<size_t>(cnt, 1) * sizeof(T);
    hipError_t e = hipMalloc((void**)&p, bytes);
    if (e != hipSuccess) { p = nullptr; return e; }
    n = cnt;
    return hipSuccess;
  }
};

enum : int { ST_ASSEMBLED = 1, ST_ANALYZED = 2, ST_FACTORED = 4, ST_SOLVED = 8 };

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};   // device address of `scratch` per device

struct HostList {  // a launch list before upload
  int64_t f_off = 0, p_off = 0;
  int64_t m_off = -1;   // offset of the work-group map, -1 if the list has none
  int64_t a_off = -1;   // offset of the per-front aux pairs, -1 if the list has none
  int32_t count = 0;
  int64_t total = 0;
  double flops = 0.0;   // algorithmic flops of the launch
  double elems = 0.0;   // algorithmic element traffic of the launch (x sizeof(T) = bytes)
};

// kernel classes of the per-launch profiler
enum KClass : int {
  KC_ASSEMBLE = 0, KC_EQUIL, KC_ZERO, KC_SCATTER, KC_EXTEND, KC_POTRF, KC_TRSM, KC_UPDATE,
  KC_SYRK, KC_COPYL, KC_LOGDET, KC_FWD, KC_BWD, KC_RESID, KC_PERMUTE, KC_SEL_GATHER, KC_SEL_Y,
  KC_SEL_GEMM, KC_SEL_DIAG, KC_SEL_OUT, KC_SEL_RED, KC_SEL_GEMM_S, KC_SYRK_S, KC_COUNT
};
const char* const kClassNames[KC_COUNT] = {
  "assemble", "equilibrate", "front_zero", "front_scatter", "extend_add", "potrf_diag", "trsm_panel",
  "update_panel", "syrk_update", "copy_L", "logdet", "solve_fwd", "solve_bwd", "residual",
  "permute", "sel_gather", "sel_Y", "sel_gemm", "sel_diag", "sel_extract", "sel_reduce", "sel_gemm_small",
  "syrk_small"};

struct Level {
  std::vector<int32_t> fronts;     // sorted by column count p descending
  int nsteps = 0;
  int64_t map_begin = 0, map_end = 0;
  HostList all;                    // every front, one work-group each
  std::vector<HostList> ext;       // extend-add per child slot (tiles = child u)
  std::vector<HostList> fvec_ext;  // vector extend-add per child slot (1 per parent)
  std::vector<HostList> potrf, trsm, upd, upd_out;   // per 64-block step
  HostList syrk, copyL, inv256;
  HostList zlow;                           // lower triangles of the fronts, 4 columns per work-group
  HostList sgather;
  int nsteps2 = 0;                                // 256-wide outer blocks of the widest front
  std::vector<HostList> fblk, fout, bpart, bblk;  // solves per outer block
  std::vector<HostList> sY2, sgemm2, sgred, spart2, sfin2;
  std::vector<HostList> sgemm4, sgred4;   // FP32: 256 x 256 tiles of the Sigma[R', K] products
  std::vector<HostList> sgemm2s;          // FP32: the same products of small fronts, 128 x 128 tiles
  HostList syrk3;                          // FP32: 256 x 256 tiles of the trailing SYRK
  HostList syrk_s;                         // FP32: the SYRK of small update matrices, 128 x 128 tiles
  std::vector<HostList> pupd4, pred4;      // FP32: left-looking panel update per outer block
  double wsize_elems_scatter = 0.0;
  // level-fused solves (one right-hand side): task ranges in the uploaded task array
  int64_t ftask_off = 0, ftask_cnt = 0;   // forward: (front, 64-row chunk), chunk-major
  int64_t btask_off = 0, btask_cnt = 0;   // backward: (front, pivot chunk), from the right
  double fbytes = 0.0, bbytes = 0.0;      // elements of L each pass reads at this depth
};

}  // namespace

struct gmrf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  int state = 0;
  int64_t n = 0, m = 0, nnzq = 0, nnza = 0;
  std::vector<int64_t> qrp, arp;
  std::vector<int32_t> qci, aci;
  int64_t nblocks = 1;
  std::vector<int64_t> block_ptr;
  bool has_b = false, has_mu = false;

  DevArr<int64_t> d_qrp, d_qdiag, d_arp, d_atp, d_cptr;
  DevArr<int32_t> d_qci, d_qrow, d_aci, d_arow, d_ati, d_cpair;
  DevArr<double> d_qval, d_aval, d_qeps, d_y, d_b, d_mu, d_qpost, d_h, d_rvec, d_qhat, d_scale;
  DevArr<int32_t> d_sexp;

  Symbolic sym;
  AnalyzeOptions opt;
  DevArr<int32_t> d_perm, d_sfirst, d_rows, d_relpos, d_child_ptr, d_child_idx, d_sparent;
  DevArr<int64_t> d_rowptr, d_Loff, d_Woff, d_Doff, d_Voff;
  DevArr<int64_t> d_map_e, d_map_off;
  DevArr<int32_t> d_lfronts;
  DevArr<int64_t> d_lprefix;
  DevArr<int2> d_wgmap;
  DevArr<int32_t> d_aux;
  DevArr<int64_t> d_bptr, d_D2off;
  int64_t D2size = 0;
  DevArr<int32_t> d_bpiv;
  std::vector<Level> levels;
  int64_t max_front = 0;
  int64_t part_max = 0;   // largest split-K partial launch (work-groups)
  int64_t gpart_max = 0;  // largest split Sigma[R', K] launch (work-groups of 128 x 128)
  int64_t gpart3_max = 0; // same for the FP32 256 x 128 tiles
  int64_t bpart_max = 0;  // largest backward-solve partial launch (work-groups)
  // level-fused solves: task lists, and the synchronisation words
  // [prog: one per supernode][tickets: 2 per depth][wait-limit error flag]
  DevArr<int2> d_tasks;
  DevArr<int32_t> d_sync;
  int64_t sync_reset = 0;   // words cleared before each pass (prog + tickets)
  // whole-forest solves: task lists (forward deepest first, backward roots first), the
  // children's update gather map and the update parts of all fronts
  DevArr<int2> d_ftasks, d_btasks;
  DevArr<double> d_cgpart;             // partial sums of the fused Jacobi CG iteration
  DevArr<int32_t> d_fgrp, d_bgrp;   // task groups of the whole-forest solves
  int64_t n_fgrp = 0, n_bgrp = 0;   // group counts (the arrays may be larger after a re-analysis)
  DevArr<int32_t> d_fneed;
  DevArr<int64_t> d_froff, d_fgptr, d_fgsrc, d_fuoff;
  DevArr<double> d_fU;

  int prec = -1;
  DevArr<char> d_L, d_D, d_D2, d_D2T, d_W0, d_W1, d_Y, d_part, d_gpart;
  DevArr<double> d_piv, d_V0, d_V1, d_xp, d_w, d_r, d_red, d_norm, d_ld, d_mu_post, d_bpart;
  DevArr<int32_t> d_status;
  int refine_iters = 0;
  double refine_resid = 0.0;
  int64_t failed_index = -1;
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  // asynchronous selected inversion: its own stream (default priority, non-blocking),
  // ordered after the factorisation and joined by every call that writes shared buffers
  hipStream_t sel_stream = nullptr;
  hipEvent_t ev_sel_start = nullptr, ev_sel_done = nullptr;
  bool sel_inflight = false;
  double phase_ms[3] = {0, 0, 0};
  bool ev_factor = false, ev_solve = false, ev_sel = false;
  // per-launch profiler (events around every launch of a class while enabled)
  bool prof = false;
  uint32_t prof_mask = 0xffffffffu;   // kernel classes that get events while profiling
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  struct Mark { int cls; size_t e0, e1; double flops, bytes; };
  std::vector<Mark> marks;
  double cls_ms[KC_COUNT] = {0};
  double cls_flops[KC_COUNT] = {0};
  double cls_bytes[KC_COUNT] = {0};
  int64_t cls_n[KC_COUNT] = {0};
  std::vector<gmrf_launch_rec_t> recs;   // per-launch records since profiling was reset
  int tsize = 8;   // bytes per working-precision element of the current numeric phase
  // Gauss-Newton scratch
  DevArr<double> d_gn_x, d_gn_d, d_gn_tmp, d_gn_part, d_gn_quad, d_gn_sel, d_gn_rec;
  hipStream_t gn_stream = nullptr;
  hipGraphExec_t gn_exec = nullptr;   // exists only during one gmrf_gn_burgers call
  DevArr<double> d_lml;               // workspace of gmrf_lml_gradient
  DevArr<double> d_cg;                // workspace of gmrf_pcg / gmrf_sample_cg
};

namespace {

gmrf_status fail(gmrf_t h, gmrf_status code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIPCHK(h, expr)                                                                   \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail(h, _e == hipErrorOutOfMemory ? GMRF_ERR_OOM : GMRF_ERR_HIP,             \
                  std::string(#expr) + ": " + hipGetErrorString(_e));                     \
  } while (0)


hipEvent_t prof_event(gmrf_t h) {
  if (h->evused == h->evpool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->evpool.push_back(e);
  }
  return h->evpool[h->evused++];
}

// run `launch` with events around it when profiling is on
template <typename F>
void prof_launch(gmrf_t h, int cls, double flops, double elems, F launch) {
  if (!h->prof || !((h->prof_mask >> cls) & 1u)) { launch(); return; }
  const size_t i0 = h->evused;
  hipEvent_t a = prof_event(h);
  if (a) (void)hipEventRecord(a, h->stream);
  launch();
  const size_t i1 = h->evused;
  hipEvent_t b = prof_event(h);
  if (b) (void)hipEventRecord(b, h->stream);
  if (a && b) h->marks.push_back({cls, i0, i1, flops, elems * (double)h->tsize});
}

void prof_fold(gmrf_t h) {
  if (h->marks.empty()) return;
  (void)hipStreamSynchronize(h->stream);
  if (h->sel_stream) (void)hipStreamSynchronize(h->sel_stream);
  for (const auto& m : h->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->evpool[m.e0], h->evpool[m.e1]) == hipSuccess) h->cls_ms[m.cls] += ms;
    h->recs.push_back({m.cls, 0, m.flops, m.bytes, (double)ms});
    h->cls_flops[m.cls] += m.flops;
    h->cls_bytes[m.cls] += m.bytes;
    h->cls_n[m.cls] += 1;
  }
  h->marks.clear();
  h->evused = 0;
}

// host wait for an in-flight selected inversion: every call that writes or reallocates
// buffers the inversion reads (factor, front buffers, launch lists) waits for it first
hipError_t sel_sync(gmrf_t h) {
  if (!h->sel_inflight) return hipSuccess;
  h->sel_inflight = false;
  return hipEventSynchronize(h->ev_sel_done);
}

template <typename T>
hipError_t upload(DevArr<T>& d, const std::vector<T>& h, hipStream_t st) {
  hipError_t e = d.alloc(h.size());
  if (e != hipSuccess) return e;
  if (h.empty()) return hipSuccess;
  e = hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

template <typename T>
hipError_t download(std::vector<T>& h, const T* d, size_t cnt, hipStream_t st) {
  h.resize(cnt);
  if (cnt == 0) return hipSuccess;
  hipError_t e = hipMemcpyAsync(h.data(), d, cnt * sizeof(T), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
}

std::string check_csr(int64_t nr, int64_t nc, const std::vector<int64_t>& rp,
                      const std::vector<int32_t>& ci, const char* name) {
  if (rp.empty() || rp[0] != 0) return std::string(name) + ": row pointer must start at 0";
  for (int64_t r = 0; r < nr; ++r) {
    if (rp[r + 1] < rp[r]) return std::string(name) + ": row pointers decrease";
    for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
      if (ci[e] < 0 || ci[e] >= nc) return std::string(name) + ": column index out of range";
      if (e > rp[r] && ci[e] <= ci[e - 1]) return std::string(name) + ": columns not strictly increasing";
    }
  }
  return std::string();
}

int64_t find_entry(const std::vector<int64_t>& rp, const std::vector<int32_t>& ci, int64_t r, int32_t c) {
  const int32_t* b = ci.data() + rp[r];
  const int32_t* e = ci.data() + rp[r + 1];
  const int32_t* it = std::lower_bound(b, e, c);
  if (it == e || *it != c) return -1;
  return rp[r] + (it - b);
}

// ------------------------------------------------------------------ plan construction
struct Cost { double flops, elems; };

// split-K of the Sigma[R', K] products at the top of the tree: with T output tiles and
// `slots` work-groups resident at once, a launch of T*S parts takes ceil(T S / slots)
// rounds of 1/S of the work each.  Take the smallest S whose round count per unit of work
// is within 10% of the ideal T / slots (parts of at least kSplitMinK rows).
constexpr int64_t kSplitMinK = 512;
constexpr int64_t kSlots128 = 256;   // 128 x 128 tiles (FP64): one resident work-group per CU
constexpr int64_t kSlots4 = 256;     // FP32 256 x 256 tiles: one per CU
// FP32 mode: products with fewer rows than this (Sigma[R', K] with |R'| < kBig4, update
// matrices of fewer than kBig4 rows) run on 128 x 128 FP32 tiles instead of the 256 x 256
// bf16 tiles, which would be mostly padding
constexpr int64_t kBig4 = 384;
// Fronts of one launch have different K (their |R'|): pick one part length P and split
// every front's K into ceil(K / P) parts, so that all parts carry about the same work.
// P minimises rounds * (P + overhead of a partial tile) over P = Kmax / S (S = 1..128) and
// P = K_f / m for every front f (m = 1..64), with parts of at least kSplitMinK rows; the
// overhead of writing and summing a partial tile is counted as kPartCost rows of K.
constexpr int64_t kPartCost = 512;
int64_t choose_part(const std::vector<std::pair<int64_t, int64_t>>& tk, int64_t slots) {
  int64_t kmax = 1;
  for (const auto& x : tk) kmax = std::max(kmax, x.second);
  const int64_t pmin = std::min<int64_t>(kSplitMinK, kmax);
  // candidate lengths: kmax / S and, for every front, its K / m (parts of one front equal)
  std::vector<int64_t> cand;
  auto push = [&](int64_t P) {
    P = std::max<int64_t>(pmin, (P + 15) / 16 * 16);
    if (P <= kmax) cand.push_back(P);
  };
  for (int64_t S = 1; S <= 128; ++S) push((kmax + S - 1) / S);
  for (const auto& x : tk)
    for (int64_t m = 1; m <= 64; ++m) push((x.second + m - 1) / m);
  cand.push_back(kmax);
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  int64_t best = kmax;
  double best_t = 1e300;
  for (auto it = cand.rbegin(); it != cand.rend(); ++it) {   // longest first: ties keep fewer parts
    const int64_t P = *it;
    int64_t wgs = 0;
    bool split = false;
    for (const auto& x : tk) {
      const int64_t parts = std::max<int64_t>(1, (x.second + P - 1) / P);
      split = split || parts > 1;
      wgs += x.first * parts;
    }
    const double t = (double)((wgs + slots - 1) / slots) * (double)(P + (split ? kPartCost : 0));
    if (t < best_t * 0.999) {
      best_t = t;
      best = P;
    }
  }
  return best;
}

int64_t choose_split(int64_t T, int64_t slots, int64_t smax) {
  if (T <= 0 || T >= 8 * slots) return 1;
  const double ideal = (double)T / (double)slots;
  int64_t best = 1;
  double best_r = 1e300;
  for (int64_t S = 1; S <= std::max<int64_t>(1, smax); ++S) {
    const double r = (double)((T * S + slots - 1) / slots) / (double)S;
    if (r <= 1.1 * ideal) return S;
    if (r < best_r - 1e-12) { best_r = r; best = S; }
  }
  return best;
}

struct ListBuilder {
  // work-group maps beyond this many entries are not kept (kernels then search the prefix)
  static constexpr int64_t kMaxMap = int64_t(1) << 27;
  std::vector<int32_t> fronts;
  std::vector<int64_t> prefix;
  std::vector<int2> wgmap;
  std::vector<int32_t> aux;
  template <typename F>
  HostList add(const std::vector<int32_t>& cand, F tiles) {
    return add(cand, tiles, [](int32_t) { return Cost{0.0, 0.0}; });
  }
  template <typename F, typename C>
  HostList add(const std::vector<int32_t>& cand, F tiles, C cost) {
    return add(cand, tiles, cost, nullptr);
  }
  // auxf(s) -> std::pair<int32_t, int32_t> stored per listed front (two ints)
  template <typename F, typename C, typename A>
  HostList add(const std::vector<int32_t>& cand, F tiles, C cost, A auxf) {
    HostList L;
    L.f_off = (int64_t)fronts.size();
    L.p_off = (int64_t)prefix.size();
    int64_t tot = 0;
    for (int32_t s : cand) {
      int64_t t = tiles(s);
      if (t <= 0) continue;
      fronts.push_back(s);
      prefix.push_back(tot);
      tot += t;
      L.count++;
      if constexpr (!std::is_same_v<A, std::nullptr_t>) {
        if (L.count == 1) L.a_off = (int64_t)aux.size();
        const std::pair<int32_t, int32_t> a = auxf(s);
        aux.push_back(a.first);
        aux.push_back(a.second);
      }
      const Cost c = cost(s);
      L.flops += c.flops;
      L.elems += c.elems;
    }
    prefix.push_back(tot);
    L.total = tot;
    if (L.count > 1 && (int64_t)wgmap.size() + tot <= kMaxMap) {
      L.m_off = (int64_t)wgmap.size();
      for (int32_t i = 0; i < L.count; ++i) {
        const int64_t a = prefix[L.p_off + i], b = prefix[L.p_off + i + 1];
        for (int64_t w = a; w < b; ++w) wgmap.push_back(make_int2(i, (int)(w - a)));
      }
    }
    return L;
  }
};

LaunchList dev_list(const gmrf_ctx* h, const HostList& L) {
  LaunchList d;
  d.fronts = h->d_lfronts.p + L.f_off;
  d.prefix = h->d_lprefix.p + L.p_off;
  d.wgmap = L.m_off >= 0 ? h->d_wgmap.p + L.m_off : nullptr;
  d.aux = L.a_off >= 0 ? h->d_aux.p + L.a_off : nullptr;
  d.count = L.count;
  d.total = L.total;
  return d;
}

DevSym dev_sym(const gmrf_ctx* h) {
  DevSym S;
  S.n = h->n;
  S.perm = h->d_perm.p;
  S.sfirst = h->d_sfirst.p;
  S.rowptr = h->d_rowptr.p;
  S.rows = h->d_rows.p;
  S.relpos = h->d_relpos.p;
  S.child_ptr = h->d_child_ptr.p;
  S.child_idx = h->d_child_idx.p;
  S.Loff = h->d_Loff.p;
  S.Woff = h->d_Woff.p;
  S.Doff = h->d_Doff.p;
  S.Voff = h->d_Voff.p;
  return S;
}

// update region of the two-level blocked panel / SYRK updates (mirrors the device side)
void upd_region(int mode, int64_t step, int64_t n, int64_t p, int64_t& clo, int64_t& chi, int64_t& klo,
                int64_t& khi) {
  const int64_t sub = kNB2 / kNB;
  if (mode == 2) { clo = p; chi = n; klo = 0; khi = p; return; }
  if (mode == 1) {
    const int64_t k2 = (step / sub) * kNB2;
    clo = k2 + kNB2; chi = p; klo = k2; khi = k2 + kNB2;
    return;
  }
  const int64_t k0 = step * kNB, kb = std::min<int64_t>(kNB, p - k0);
  const int64_t oe = std::min<int64_t>((step / sub + 1) * kNB2, p);
  clo = k0 + kb; chi = oe; klo = k0; khi = k0 + kb;
}

int64_t upd_tiles(int64_t n, int64_t p, int mode, int64_t step, int64_t ts, int64_t tr = 0) {
  int64_t clo, chi, klo, khi;
  upd_region(mode, step, n, p, clo, chi, klo, khi);
  if (tr <= 0) tr = ts;   // tile rows (default: square tiles)
  int64_t t = 0;
  for (int64_t c0 = clo; c0 < chi; c0 += ts) t += (n - c0 + tr - 1) / tr;
  return t;
}

Cost upd_cost(int64_t n, int64_t p, int mode, int64_t step) {
  int64_t clo, chi, klo, khi;
  upd_region(mode, step, n, p, clo, chi, klo, khi);
  // lower-trapezoid entries: sum over columns c of (n - c)
  const double cols = (double)std::max<int64_t>(chi - clo, 0);
  const double E = cols * (double)(n - clo) - 0.5 * cols * (cols - 1.0);
  const double K = (double)(khi - klo);
  return Cost{2.0 * K * E, 2.0 * E + (double)(n - clo) * K};
}

gmrf_status build_plan(gmrf_t h) {
  const Symbolic& Y = h->sym;
  const int nb = kNB;
  h->levels.assign(Y.max_depth + 1, Level());
  h->max_front = 0;
  for (int32_t s = 0; s < Y.ns; ++s) {
    h->levels[Y.depth[s]].fronts.push_back(s);
    h->max_front = std::max<int64_t>(h->max_front, Y.nf(s));
  }
  // scatter / gather map: every stored entry of Q, grouped by depth of the owning front
  std::vector<int32_t> colsup(h->n);
  for (int32_t s = 0; s < Y.ns; ++s)
    for (int32_t j = Y.sfirst[s]; j < Y.sfirst[s + 1]; ++j) colsup[j] = s;
  std::vector<int64_t> cnt(Y.max_depth + 2, 0);
  std::vector<int32_t> edep(h->nnzq);
  std::vector<int64_t> eoff(h->nnzq);
  for (int64_t r = 0; r < h->n; ++r) {
    for (int64_t e = h->qrp[r]; e < h->qrp[r + 1]; ++e) {
      const int32_t i = Y.iperm[r], j = Y.iperm[h->qci[e]];
      const int32_t lo = std::min(i, j), hi = std::max(i, j);
      const int32_t s = colsup[lo];
      const int32_t* rb = Y.rows.data() + Y.rowptr[s];
      const int32_t* re = Y.rows.data() + Y.rowptr[s + 1];
      const int32_t* it = std::lower_bound(rb, re, hi);
      if (it == re || *it != hi) return fail(h, GMRF_ERR_ARG, "internal: entry of Q outside the symbolic factor");
      const int64_t nf = Y.nf(s);
      eoff[e] = Y.Woff[s] + (int64_t)(it - rb) + (int64_t)(lo - Y.sfirst[s]) * nf;
      edep[e] = Y.depth[s];
      cnt[Y.depth[s] + 1]++;
    }
  }
  for (int d = 0; d <= Y.max_depth; ++d) cnt[d + 1] += cnt[d];
  std::vector<int64_t> map_e(h->nnzq), map_off(h->nnzq);
  {
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t r = 0; r < h->n; ++r) {
      for (int64_t e = h->qrp[r]; e < h->qrp[r + 1]; ++e) {
        const int32_t i = Y.iperm[r], j = Y.iperm[h->qci[e]];
        const int64_t q = fill[edep[e]]++;
        map_e[q] = i >= j ? e : -(e + 1);
        map_off[q] = eoff[e];
      }
    }
  }
  edep.clear(); edep.shrink_to_fit(); eoff.clear(); eoff.shrink_to_fit();

  ListBuilder B;
  h->part_max = 0;
  h->gpart_max = 0;
  h->gpart3_max = 0;
  h->bpart_max = 0;
  for (int d = 0; d <= Y.max_depth; ++d) {
    Level& lv = h->levels[d];
    lv.map_begin = cnt[d];
    lv.map_end = cnt[d + 1];
    std::stable_sort(lv.fronts.begin(), lv.fronts.end(),
                     [&](int32_t a, int32_t b) { return Y.p(a) > Y.p(b); });
    lv.nsteps = 0;
    int maxch = 0;
    for (int32_t s : lv.fronts) {
      lv.nsteps = std::max(lv.nsteps, (Y.p(s) + nb - 1) / nb);
      maxch = std::max(maxch, Y.child_ptr[s + 1] - Y.child_ptr[s]);
    }
    auto nF = [&](int32_t s) { return (int64_t)Y.nf(s); };
    auto pF = [&](int32_t s) { return (int64_t)Y.p(s); };
    // fronts of at most kNB rows are factored whole by the diagonal-block kernel
    auto small = [&](int32_t s) { return nF(s) <= (int64_t)kNB; };
    lv.all = B.add(lv.fronts, [](int32_t) { return (int64_t)1; },
                   [&](int32_t s) { return Cost{0.0, (double)pF(s) + (double)nF(s)}; });
    for (int c = 0; c < maxch; ++c) {
      auto child = [&](int32_t s) { return Y.child_idx[Y.child_ptr[s] + c]; };
      auto has = [&](int32_t s) { return Y.child_ptr[s + 1] - Y.child_ptr[s] > c; };
      lv.ext.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        return has(s) ? (nF(child(s)) - pF(child(s)) + kExtCols - 1) / kExtCols : 0;
      }, [&](int32_t s) {
        const double u = (double)(nF(child(s)) - pF(child(s)));
        return Cost{0.5 * u * (u + 1), 1.5 * u * (u + 1)};
      }));
      lv.fvec_ext.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return has(s) ? 1 : 0; }));
    }
    for (int k = 0; k < lv.nsteps; ++k) {
      const int64_t k0 = (int64_t)k * nb;
      auto active = [&](int32_t s) { return pF(s) > k0; };
      auto kb = [&](int32_t s) { return std::min<int64_t>(nb, pF(s) - k0); };
      auto below = [&](int32_t s) { return (double)(nF(s) - k0 - kb(s)); };
      lv.potrf.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return active(s) ? 1 : 0; },
                               [&](int32_t s) {
                                 const double b3 = (double)kb(s);
                                 if (small(s)) {
                                   const double r = below(s), nn = (double)nF(s);
                                   const Cost u = nF(s) > pF(s) ? upd_cost(nF(s), pF(s), 2, 0) : Cost{0.0, 0.0};
                                   return Cost{2.0 * b3 * b3 * b3 / 3.0 + r * b3 * b3 + u.flops,
                                               nn * (nn + 1.0) + b3 * b3};
                                 }
                                 return Cost{2.0 * b3 * b3 * b3 / 3.0, 3.0 * b3 * b3};
                               }));
      lv.trsm.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        if (!active(s) || small(s)) return 0;
        const int64_t rows = nF(s) - k0 - kb(s);
        return (rows + kTile - 1) / kTile;
      }, [&](int32_t s) {
        const double r = below(s), b = (double)kb(s);
        return Cost{r * b * b, 2.0 * r * b + b * b};
      }));
      lv.upd.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        if (!active(s) || small(s)) return 0;
        return upd_tiles(nF(s), pF(s), 0, k, kTile);
      }, [&](int32_t s) { return upd_cost(nF(s), pF(s), 0, k); }));
      const bool outer_here = (k + 1) % (kNB2 / nb) == 0;
      lv.upd_out.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        if (!outer_here || pF(s) <= (int64_t)(k + 1) * nb) return 0;
        return upd_tiles(nF(s), pF(s), 1, k, kBigTile);
      }, [&](int32_t s) { return upd_cost(nF(s), pF(s), 1, k); }));
    }
    // FP32 left-looking panel updates, one per outer block K >= 1 (list K-1 unused for K = 0)
    {
      int nK = 0;
      for (int32_t s : lv.fronts) nK = std::max<int>(nK, (int)((pF(s) + kNB2 - 1) / kNB2));
      lv.pupd4.assign(std::max(nK, 1), HostList());
      lv.pred4.assign(std::max(nK, 1), HostList());
      for (int K = 1; K < nK; ++K) {
        const int64_t k2 = (int64_t)K * kNB2;
        auto pact = [&](int32_t s) { return pF(s) > k2; };
        auto pkb2 = [&](int32_t s) { return std::min<int64_t>(kNB2, pF(s) - k2); };
        auto ptiles = [&](int32_t s) -> int64_t { return pact(s) ? (nF(s) - k2 + 255) / 256 : 0; };
        int64_t ptot = 0;
        for (int32_t s : lv.fronts) ptot += ptiles(s);
        const int64_t pS = choose_split(ptot, kSlots4, k2 / kSplitMinK);
        auto psplit = [&](int32_t s) -> int64_t { return ptiles(s) > 0 ? std::max<int64_t>(1, pS) : 1; };
        lv.pupd4[K] = B.add(lv.fronts, [&](int32_t s) -> int64_t { return ptiles(s) * psplit(s); },
                            [&](int32_t s) {
          const double b = (double)pkb2(s), m = (double)(nF(s) - k2);
          const double E = b * m - 0.5 * b * (b - 1.0);
          return Cost{2.0 * (double)k2 * E, 2.0 * E + (m + b) * (double)k2};
        }, [&](int32_t s) { return std::make_pair((int32_t)psplit(s), (int32_t)0); });
        const HostList& G = lv.pupd4[K];
        std::unordered_map<int32_t, int64_t> gbase;
        for (int32_t i = 0; i < G.count; ++i) gbase[B.fronts[G.f_off + i]] = B.prefix[G.p_off + i];
        if (pS > 1) h->gpart3_max = std::max(h->gpart3_max, 2 * G.total);   // 256 x 128 units
        lv.pred4[K] = B.add(lv.fronts, [&](int32_t s) -> int64_t { return psplit(s) > 1 ? 4 * ptiles(s) : 0; },
                            [&](int32_t s) {
          const double b = (double)pkb2(s), m = (double)(nF(s) - k2);
          return Cost{0.0, (double)psplit(s) * m * b + 2.0 * m * b};
        }, [&](int32_t s) { return std::make_pair((int32_t)psplit(s), (int32_t)gbase[s]); });
      }
    }
    // two-level selected inversion: outer blocks of 256 columns, counted from the right
    lv.nsteps2 = 0;
    for (int32_t s : lv.fronts) lv.nsteps2 = std::max<int>(lv.nsteps2, (int)((pF(s) + kNB2 - 1) / kNB2));
    for (int t = 0; t < lv.nsteps2; ++t) {
      auto oK = [&](int32_t s) { return (pF(s) + kNB2 - 1) / kNB2 - 1 - t; };
      auto oact = [&](int32_t s) { return oK(s) >= 0; };
      auto okb2 = [&](int32_t s) { return std::min<int64_t>(kNB2, pF(s) - oK(s) * kNB2); };
      auto otail = [&](int32_t s) { return nF(s) - oK(s) * kNB2 - okb2(s); };
      auto onsub = [&](int32_t s) { return (okb2(s) + nb - 1) / nb; };
      auto onct = [&](int32_t s) { return (okb2(s) + kBigTile - 1) / kBigTile; };
      lv.sY2.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        return oact(s) ? ((otail(s) + kBigTile - 1) / kBigTile) * onct(s) : 0;
      }, [&](int32_t s) {
        const double r = (double)otail(s), b = (double)okb2(s);
        return Cost{r * b * b, 2.0 * r * b + b * b};
      }));
      // Sigma[R', K] = -Sigma[R', R'] Y: 128 x 128 output tiles; when a depth has too few
      // tiles to fill the chip (top of the tree), the long K = |R'| is split into parts
      // whose partial tiles a second launch adds in a fixed order
      auto gtiles = [&](int32_t s) -> int64_t {
        return oact(s) ? ((otail(s) + kBigTile - 1) / kBigTile) * onct(s) : 0;
      };
      int64_t gtot = 0;
      for (int32_t s : lv.fronts) gtot += gtiles(s);
      int64_t gmaxk = 0;
      for (int32_t s : lv.fronts) if (gtiles(s) > 0) gmaxk = std::max<int64_t>(gmaxk, otail(s) / kSplitMinK);
      const int64_t gS = choose_split(gtot, kSlots128, gmaxk);
      auto gsplit = [&](int32_t s) -> int64_t {
        if (gtiles(s) == 0) return 1;
        return std::max<int64_t>(1, std::min<int64_t>(gS, otail(s) / kSplitMinK));
      };
      lv.sgemm2.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return gtiles(s) * gsplit(s); },
                                [&](int32_t s) {
        const double r = (double)otail(s), b = (double)okb2(s);
        return Cost{2.0 * r * r * b, r * r + 3.0 * r * b};
      }, [&](int32_t s) { return std::make_pair((int32_t)gsplit(s), (int32_t)0); }));
      {
        const HostList& G = lv.sgemm2.back();
        std::unordered_map<int32_t, int64_t> gbase;
        bool any = false;
        for (int32_t i = 0; i < G.count; ++i) gbase[B.fronts[G.f_off + i]] = B.prefix[G.p_off + i];
        for (int32_t s : lv.fronts) any = any || gsplit(s) > 1;
        if (any) h->gpart_max = std::max(h->gpart_max, G.total);
        lv.sgred.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return gsplit(s) > 1 ? 2 * gtiles(s) : 0; },
                                 [&](int32_t s) {
          const double r = (double)otail(s), b = (double)okb2(s);
          return Cost{0.0, (double)gsplit(s) * r * b + 2.0 * r * b};
        }, [&](int32_t s) { return std::make_pair((int32_t)gsplit(s), (int32_t)gbase[s]); }));
      }
      {
        // FP32 variant: 256 x 256 tiles (one work-group per 256 rows of R' and K part), one
        // resident work-group per CU.  When every product of the launch has fewer than kBig4
        // rows (most of a 256 x 256 tile would be padding) they take the 128 x 128 FP32 tiles
        // instead, unsplit; a launch with larger products keeps them all on the 256 x 256
        // tiles, whose split-K choice covers the whole launch
        bool any_big = false;
        for (int32_t s : lv.fronts) any_big = any_big || (oact(s) && otail(s) >= kBig4);
        auto big4 = [&](int32_t) { return any_big; };
        auto gtiles4 = [&](int32_t s) -> int64_t { return oact(s) && big4(s) ? (otail(s) + 255) / 256 : 0; };
        lv.sgemm2s.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return big4(s) ? 0 : gtiles(s); },
                                   [&](int32_t s) {
          const double r = (double)otail(s), b = (double)okb2(s);
          return Cost{2.0 * r * r * b, r * r + 3.0 * r * b};
        }, [&](int32_t) { return std::make_pair((int32_t)1, (int32_t)0); }));
        std::vector<std::pair<int64_t, int64_t>> tk4;
        for (int32_t s : lv.fronts)
          if (gtiles4(s) > 0) tk4.emplace_back(gtiles4(s), otail(s));
        const int64_t gP4 = choose_part(tk4, kSlots4);
        auto gsplit4 = [&](int32_t s) -> int64_t {
          if (gtiles4(s) == 0) return 1;
          return std::max<int64_t>(1, (otail(s) + gP4 - 1) / gP4);
        };
        lv.sgemm4.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return gtiles4(s) * gsplit4(s); },
                                  [&](int32_t s) {
          const double r = (double)otail(s), b = (double)okb2(s);
          return Cost{2.0 * r * r * b, r * r + 3.0 * r * b};
        }, [&](int32_t s) { return std::make_pair((int32_t)gsplit4(s), (int32_t)0); }));
        const HostList& G = lv.sgemm4.back();
        std::unordered_map<int32_t, int64_t> gbase;
        bool any = false;
        for (int32_t i = 0; i < G.count; ++i) gbase[B.fronts[G.f_off + i]] = B.prefix[G.p_off + i];
        for (int32_t s : lv.fronts) any = any || gsplit4(s) > 1;
        if (any) h->gpart3_max = std::max(h->gpart3_max, 2 * G.total);   // 256 x 128 units
        lv.sgred4.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
          return gsplit4(s) > 1 ? 4 * gtiles4(s) : 0;
        }, [&](int32_t s) {
          const double r = (double)otail(s), b = (double)okb2(s);
          return Cost{0.0, (double)gsplit4(s) * r * b + 2.0 * r * b};
        }, [&](int32_t s) { return std::make_pair((int32_t)gsplit4(s), (int32_t)gbase[s]); }));
      }
      lv.spart2.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        return oact(s) ? std::max<int64_t>(1, (otail(s) + kSelChunk - 1) / kSelChunk) * onsub(s) * onsub(s) : 0;
      }, [&](int32_t s) {
        // the symmetric block's lower half (the kernel computes its lower 64x64 tiles)
        const double r = (double)otail(s), b = (double)okb2(s);
        return Cost{r * b * (b + 1.0), 2.0 * r * b};
      }));
      h->part_max = std::max(h->part_max, lv.spart2.back().total);
      // solves: forward outer block t (left to right), backward outer block from the right
      auto fact = [&](int32_t s) { return pF(s) > (int64_t)t * kNB2; };
      auto fkb2 = [&](int32_t s) { return std::min<int64_t>(kNB2, pF(s) - (int64_t)t * kNB2); };
      auto fbelow = [&](int32_t s) { return nF(s) - (int64_t)t * kNB2 - fkb2(s); };
      lv.fblk.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return fact(s) ? (fkb2(s) + 63) / 64 : 0; },
                              [&](int32_t s) { const double b = (double)fkb2(s); return Cost{b * b, 0.5 * b * b}; }));
      lv.fout.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        return fact(s) ? (fbelow(s) + 63) / 64 : 0;
      }, [&](int32_t s) {
        const double r = (double)fbelow(s), b = (double)fkb2(s);
        return Cost{2.0 * r * b, r * b};
      }));
      lv.bpart.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t {
        return oact(s) ? std::max<int64_t>(1, (otail(s) + 255) / 256) : 0;
      }, [&](int32_t s) {
        const double r = (double)otail(s), b = (double)okb2(s);
        return Cost{2.0 * r * b, r * b};
      }));
      h->bpart_max = std::max(h->bpart_max, lv.bpart.back().total);
      lv.bblk.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return oact(s) ? (okb2(s) + 63) / 64 : 0; },
                              [&](int32_t s) { const double b = (double)okb2(s); return Cost{b * b, 0.5 * b * b}; }));
      lv.sfin2.push_back(B.add(lv.fronts, [&](int32_t s) -> int64_t { return oact(s) ? onsub(s) * onsub(s) : 0; },
                               [&](int32_t s) { const double b = (double)okb2(s); return Cost{b * b * b / 3.0, 2.0 * b * b}; }));
    }
    lv.syrk = B.add(lv.fronts, [&](int32_t s) -> int64_t {
      return nF(s) > pF(s) && !small(s) ? upd_tiles(nF(s), pF(s), 2, 0, kBigTile) : 0;
    }, [&](int32_t s) { return small(s) ? Cost{0.0, 0.0} : upd_cost(nF(s), pF(s), 2, 0); });
    // FP32 SYRK: the 128 x 128 FP32 tiles when every update matrix of the depth has fewer
    // than kBig4 rows, else all on the 256 x 256 tiles
    bool any_big_u = false;
    for (int32_t s : lv.fronts) any_big_u = any_big_u || (!small(s) && nF(s) - pF(s) >= kBig4);
    auto big_syrk = [&](int32_t) { return any_big_u; };
    lv.syrk3 = B.add(lv.fronts, [&](int32_t s) -> int64_t {
      return nF(s) > pF(s) && !small(s) && big_syrk(s) ? upd_tiles(nF(s), pF(s), 2, 0, 256, 256) : 0;
    }, [&](int32_t s) { return small(s) || !big_syrk(s) ? Cost{0.0, 0.0} : upd_cost(nF(s), pF(s), 2, 0); });
    lv.syrk_s = B.add(lv.fronts, [&](int32_t s) -> int64_t {
      return nF(s) > pF(s) && !small(s) && !big_syrk(s) ? upd_tiles(nF(s), pF(s), 2, 0, kBigTile) : 0;
    }, [&](int32_t s) { return small(s) || big_syrk(s) ? Cost{0.0, 0.0} : upd_cost(nF(s), pF(s), 2, 0); });
    lv.inv256 = B.add(lv.fronts, [&](int32_t s) -> int64_t { return (pF(s) + nb - 1) / nb; }, [&](int32_t s) {
      const double p = (double)pF(s);
      return Cost{p * (double)kNB2 * (double)kNB2 / 3.0, p * (double)kNB2};
    });
    lv.zlow = B.add(lv.fronts, [&](int32_t s) -> int64_t { return (nF(s) + 3) / 4; }, [&](int32_t s) {
      const double n = (double)nF(s);
      return Cost{0.0, 0.5 * n * (n + 1.0)};
    });
    lv.copyL = B.add(lv.fronts, [&](int32_t s) -> int64_t { return pF(s); }, [&](int32_t s) {
      const double p = (double)pF(s), n = (double)nF(s);
      return Cost{0.0, 2.0 * (p * n - 0.5 * p * (p - 1.0))};
    });
    lv.sgather = B.add(lv.fronts, [&](int32_t s) -> int64_t {
      return Y.sparent[s] >= 0 ? (nF(s) - pF(s) + kExtCols - 1) / kExtCols : 0;
    }, [&](int32_t s) { const double u = (double)(nF(s) - pF(s)); return Cost{0.0, 2.0 * u * u}; });
    lv.wsize_elems_scatter = (double)(lv.map_end - lv.map_begin);
  }
  // level-fused solve tasks: forward chunk-major over the depth's fronts, backward pivot
  // chunks from the right; each task follows every task it waits for
  {
    std::vector<int2> tasks;
    for (int d = 0; d <= Y.max_depth; ++d) {
      Level& lv = h->levels[d];
      int cmax = 0, pmax = 0;
      for (int32_t s : lv.fronts) {
        cmax = std::max<int>(cmax, (int)((Y.nf(s) + 63) / 64));
        pmax = std::max<int>(pmax, (int)((Y.p(s) + 63) / 64));
      }
      lv.ftask_off = (int64_t)tasks.size();
      lv.fbytes = 0.0;
      for (int c = 0; c < cmax; ++c)
        for (int32_t s : lv.fronts)
          if (c * 64 < Y.nf(s)) tasks.push_back(make_int2(s, c));
      lv.ftask_cnt = (int64_t)tasks.size() - lv.ftask_off;
      lv.btask_off = (int64_t)tasks.size();
      for (int k = 0; k < pmax; ++k)
        for (int32_t s : lv.fronts) {
          const int P = (int)((Y.p(s) + 63) / 64);
          if (k < P) tasks.push_back(make_int2(s, P - 1 - k));
        }
      lv.btask_cnt = (int64_t)tasks.size() - lv.btask_off;
      for (int32_t s : lv.fronts) {
        const double nn = (double)Y.nf(s), pp = (double)Y.p(s);
        lv.fbytes += pp * nn - 0.5 * pp * (pp - 1.0);
      }
      lv.bbytes = lv.fbytes;
    }
    HIPCHK(h, upload(h->d_tasks, tasks, h->stream));
    // sync words: [prog: ns][kids: ns][tickets: 2 per depth + 2 forest][wait-limit flag]
    h->sync_reset = 2 * (int64_t)Y.ns + 2 * (int64_t)(Y.max_depth + 1) + 2;
    HIPCHK(h, h->d_sync.alloc((size_t)h->sync_reset + 1));
    launch_fill_i32(h->stream, h->d_sync.p, h->sync_reset + 1, 0);
    // whole-forest task lists: each depth's list, deepest depth first (forward) or the
    // roots first (backward); inside a depth the order of the level lists above
    std::vector<int2> ft, bt;
    for (int d = Y.max_depth; d >= 0; --d) {
      const Level& lv = h->levels[d];
      ft.insert(ft.end(), tasks.begin() + lv.ftask_off, tasks.begin() + lv.ftask_off + lv.ftask_cnt);
    }
    for (int d = 0; d <= Y.max_depth; ++d) {
      const Level& lv = h->levels[d];
      bt.insert(bt.end(), tasks.begin() + lv.btask_off, tasks.begin() + lv.btask_off + lv.btask_cnt);
    }
    // update parts, children's gather map (rows of every front; children in ascending
    // slot order, then their update rows in order), and per-front child chunk counts
    std::vector<int64_t> uoff(Y.ns + 1, 0), roff(Y.ns + 1, 0);
    for (int32_t s2 = 0; s2 < Y.ns; ++s2) {
      uoff[s2 + 1] = uoff[s2] + (Y.nf(s2) - Y.p(s2));
      roff[s2 + 1] = roff[s2] + Y.nf(s2);
    }
    std::vector<int64_t> gptr(roff[Y.ns] + 1, 0);
    std::vector<int32_t> need(Y.ns, 0);
    for (int32_t s2 = 0; s2 < Y.ns; ++s2) {
      for (int32_t k = Y.child_ptr[s2]; k < Y.child_ptr[s2 + 1]; ++k) {
        const int32_t ch = Y.child_idx[k];
        const int64_t pc = Y.p(ch), nc = Y.nf(ch);
        for (int64_t a = pc; a < nc; ++a) gptr[roff[s2] + Y.relpos[Y.rowptr[ch] + a] + 1]++;
        if (nc > pc) need[s2] += (int32_t)((nc + 63) / 64 - pc / 64);
      }
    }
    for (size_t i = 0; i + 1 < gptr.size(); ++i) gptr[i + 1] += gptr[i];
    std::vector<int64_t> gsrc(gptr.back());
    {
      std::vector<int64_t> fill(gptr.begin(), gptr.end() - 1);
      for (int32_t s2 = 0; s2 < Y.ns; ++s2)
        for (int32_t k = Y.child_ptr[s2]; k < Y.child_ptr[s2 + 1]; ++k) {
          const int32_t ch = Y.child_idx[k];
          const int64_t pc = Y.p(ch), nc = Y.nf(ch);
          for (int64_t a = pc; a < nc; ++a)
            gsrc[fill[roff[s2] + Y.relpos[Y.rowptr[ch] + a]]++] = uoff[ch] + (a - pc);
        }
    }
    // task groups: up to 16 consecutive tasks of fronts with at most 256 rows share a
    // work-group; a task of a larger front is a group of its own
    auto groups = [&](const std::vector<int2>& tl) {
      std::vector<int32_t> g{0};
      int run = 0;
      for (size_t i = 0; i < tl.size(); ++i) {
        const bool small = Y.nf(tl[i].x) <= 256;
        if (i > 0 && (!small || run == 16 || Y.nf(tl[i - 1].x) > 256)) {
          g.push_back((int32_t)i);
          run = 0;
        }
        ++run;
      }
      g.push_back((int32_t)tl.size());
      if (tl.empty()) g.assign(1, 0);
      return g;
    };
    const std::vector<int32_t> fg = groups(ft), bg = groups(bt);
    HIPCHK(h, upload(h->d_ftasks, ft, h->stream));
    HIPCHK(h, upload(h->d_btasks, bt, h->stream));
    HIPCHK(h, upload(h->d_fgrp, fg, h->stream));
    HIPCHK(h, upload(h->d_bgrp, bg, h->stream));
    h->n_fgrp = (int64_t)fg.size() - 1;
    h->n_bgrp = (int64_t)bg.size() - 1;
    HIPCHK(h, upload(h->d_fneed, need, h->stream));
    HIPCHK(h, upload(h->d_froff, roff, h->stream));
    HIPCHK(h, upload(h->d_fgptr, gptr, h->stream));
    HIPCHK(h, upload(h->d_fgsrc, gsrc, h->stream));
    HIPCHK(h, upload(h->d_fuoff, uoff, h->stream));
    HIPCHK(h, h->d_fU.alloc((size_t)std::max<int64_t>(uoff[Y.ns], 1)));
  }
  hipStream_t st = h->stream;
  HIPCHK(h, upload(h->d_lfronts, B.fronts, st));
  HIPCHK(h, upload(h->d_lprefix, B.prefix, st));
  HIPCHK(h, upload(h->d_wgmap, B.wgmap, st));
  HIPCHK(h, upload(h->d_aux, B.aux, st));
  HIPCHK(h, upload(h->d_map_e, map_e, st));
  HIPCHK(h, upload(h->d_map_off, map_off, st));
  HIPCHK(h, upload(h->d_perm, Y.perm, st));
  HIPCHK(h, upload(h->d_sfirst, Y.sfirst, st));
  HIPCHK(h, upload(h->d_rowptr, Y.rowptr, st));
  HIPCHK(h, upload(h->d_rows, Y.rows, st));
  HIPCHK(h, upload(h->d_relpos, Y.relpos, st));
  HIPCHK(h, upload(h->d_child_ptr, Y.child_ptr, st));
  HIPCHK(h, upload(h->d_child_idx, Y.child_idx, st));
  HIPCHK(h, upload(h->d_sparent, Y.sparent, st));
  HIPCHK(h, upload(h->d_Loff, Y.Loff, st));
  HIPCHK(h, upload(h->d_Woff, Y.Woff, st));
  HIPCHK(h, upload(h->d_Doff, Y.Doff, st));
  HIPCHK(h, upload(h->d_Voff, Y.Voff, st));
  // storage of the 256-wide inverse diagonal blocks (selected inversion)
  {
    std::vector<int64_t> d2(Y.ns, 0);
    int64_t off = 0;
    for (int32_t s = 0; s < Y.ns; ++s) {
      const int64_t p = Y.p(s), nK = (p + kNB2 - 1) / kNB2, last = p - (nK - 1) * kNB2;
      d2[s] = off;
      off += (nK - 1) * (int64_t)kNB2 * kNB2 + last * last;
    }
    h->D2size = off;
    HIPCHK(h, upload(h->d_D2off, d2, st));
  }
  // per-block pivot lists for the log-determinant
  {
    std::vector<int64_t> bp(h->nblocks + 1, 0);
    std::vector<int32_t> owner(h->n);
    for (int64_t b = 0; b < h->nblocks; ++b)
      for (int64_t o = h->block_ptr[b]; o < h->block_ptr[b + 1]; ++o) owner[o] = (int32_t)b;
    for (int64_t j = 0; j < h->n; ++j) bp[owner[Y.perm[j]] + 1]++;
    for (int64_t b = 0; b < h->nblocks; ++b) bp[b + 1] += bp[b];
    std::vector<int32_t> bpiv(h->n);
    std::vector<int64_t> fill(bp.begin(), bp.end() - 1);
    for (int64_t j = 0; j < h->n; ++j) bpiv[fill[owner[Y.perm[j]]]++] = (int32_t)j;
    HIPCHK(h, upload(h->d_bptr, bp, st));
    HIPCHK(h, upload(h->d_bpiv, bpiv, st));
  }
  return GMRF_OK;
}

// ------------------------------------------------------------------ numeric drivers
template <typename T>
gmrf_status alloc_numeric(gmrf_t h) {
  const Symbolic& Y = h->sym;
  HIPCHK(h, h->d_L.alloc((size_t)Y.Lsize * sizeof(T)));
  HIPCHK(h, h->d_D.alloc((size_t)Y.Dsize * sizeof(T)));
  HIPCHK(h, h->d_D2.alloc((size_t)std::max<int64_t>(h->D2size, 1) * sizeof(T)));
  HIPCHK(h, h->d_D2T.alloc((size_t)std::max<int64_t>(h->D2size, 1) * sizeof(T)));
  HIPCHK(h, h->d_W0.alloc((size_t)std::max<int64_t>(Y.Wsize[0], 1) * sizeof(T)));
  HIPCHK(h, h->d_W1.alloc((size_t)std::max<int64_t>(Y.Wsize[1], 1) * sizeof(T)));
  HIPCHK(h, h->d_piv.alloc(h->n));
  HIPCHK(h, h->d_status.alloc(1));
  HIPCHK(h, h->d_scale.alloc(h->n));
  HIPCHK(h, h->d_sexp.alloc(h->n));
  HIPCHK(h, h->d_qhat.alloc(h->nnzq));
  if (std::is_same<T, float>::value)
    HIPCHK(h, h->d_gpart.alloc((size_t)std::max<int64_t>(h->gpart3_max, 1) * 256 * 128 * sizeof(float)));
  return GMRF_OK;
}

template <typename T>
gmrf_status run_factor(gmrf_t h) {
  const Symbolic& Y = h->sym;
  hipStream_t st = h->stream;
  gmrf_status rc = alloc_numeric<T>(h);
  if (rc != GMRF_OK) return rc;
  const DevSym S = dev_sym(h);
  h->tsize = (int)sizeof(T);
  prof_launch(h, KC_EQUIL, 0.0, 3.0 * h->nnzq, [&] {
    launch_equilibrate(st, h->n, h->nnzq, h->d_qdiag.p, h->d_qrow.p, h->d_qci.p, h->d_qpost.p, h->d_sexp.p,
                       h->d_scale.p, h->d_qhat.p);
  });
  launch_fill_i32(st, h->d_status.p, 1, INT_MAX);
  if (h->d_sync.p) launch_fill_i32(st, h->d_sync.p + h->sync_reset, 1, 0);   // solve wait-limit flag
  T* W[2] = {(T*)h->d_W0.p, (T*)h->d_W1.p};
  for (int d = Y.max_depth; d >= 0; --d) {
    const Level& lv = h->levels[d];
    NumBufs<T> B;
    B.L = (T*)h->d_L.p;
    B.D = (T*)h->d_D.p;
    B.piv = h->d_piv.p;
    B.Wcur = W[d & 1];
    B.Wchild = W[(d + 1) & 1];
    B.status = h->d_status.p;
    prof_launch(h, KC_ZERO, 0.0, lv.zlow.elems, [&] { launch_zero_lower<T>(st, S, dev_list(h, lv.zlow), B.Wcur); });
    prof_launch(h, KC_SCATTER, 0.0, 2.0 * lv.wsize_elems_scatter, [&] {
      launch_scatter<T>(st, lv.map_end - lv.map_begin, h->d_map_e.p + lv.map_begin,
                        h->d_map_off.p + lv.map_begin, h->d_qhat.p, B.Wcur);
    });
    for (size_t c = 0; c < lv.ext.size(); ++c)
      prof_launch(h, KC_EXTEND, lv.ext[c].flops, lv.ext[c].elems, [&] {
        launch_extend_add<T>(st, S, dev_list(h, lv.ext[c]), (int)c, B.Wchild, B.Wcur);
      });
    for (int k = 0; k < lv.nsteps; ++k) {
      if constexpr (std::is_same<T, float>::value) {
        const int K = k / (kNB2 / kNB);
        if (k % (kNB2 / kNB) == 0 && K >= 1 && K < (int)lv.pupd4.size()) {
          if (lv.pupd4[K].total > 0)
            prof_launch(h, KC_UPDATE, lv.pupd4[K].flops, lv.pupd4[K].elems, [&] {
              launch_panel_upd4(st, S, dev_list(h, lv.pupd4[K]), K, B, (float*)h->d_gpart.p);
            });
          if (lv.pred4[K].total > 0)
            prof_launch(h, KC_UPDATE, 0.0, lv.pred4[K].elems, [&] {
              launch_panel_red4(st, S, dev_list(h, lv.pred4[K]), K, B, (const float*)h->d_gpart.p);
            });
        }
      }
      prof_launch(h, KC_POTRF, lv.potrf[k].flops, lv.potrf[k].elems,
                  [&] { launch_potrf<T>(st, S, dev_list(h, lv.potrf[k]), k, B); });
      if (lv.trsm[k].total > 0)
        prof_launch(h, KC_TRSM, lv.trsm[k].flops, lv.trsm[k].elems,
                    [&] { launch_trsm<T>(st, S, dev_list(h, lv.trsm[k]), k, B); });
      if (lv.upd[k].total > 0)
        prof_launch(h, KC_UPDATE, lv.upd[k].flops, lv.upd[k].elems,
                    [&] { launch_update<T>(st, S, dev_list(h, lv.upd[k]), k, 0, B); });
      if (!std::is_same<T, float>::value && lv.upd_out[k].total > 0)
        prof_launch(h, KC_UPDATE, lv.upd_out[k].flops, lv.upd_out[k].elems,
                    [&] { launch_update<T>(st, S, dev_list(h, lv.upd_out[k]), k, 1, B); });
    }
    if constexpr (std::is_same<T, float>::value) {
      if (lv.syrk3.total > 0)
        prof_launch(h, KC_SYRK, lv.syrk3.flops, lv.syrk3.elems,
                    [&] { launch_syrk4(st, S, dev_list(h, lv.syrk3), B); });
      if (lv.syrk_s.total > 0)
        prof_launch(h, KC_SYRK_S, lv.syrk_s.flops, lv.syrk_s.elems,
                    [&] { launch_update<T>(st, S, dev_list(h, lv.syrk_s), 0, 2, B); });
    } else {
      if (lv.syrk.total > 0)
        prof_launch(h, KC_SYRK, lv.syrk.flops, lv.syrk.elems,
                    [&] { launch_update<T>(st, S, dev_list(h, lv.syrk), 0, 2, B); });
    }
    prof_launch(h, KC_POTRF, lv.inv256.flops, lv.inv256.elems, [&] {
      launch_inv256<T>(st, S, dev_list(h, lv.inv256), B.Wcur, 1, B.D, h->d_D2off.p, (T*)h->d_D2.p,
                       (T*)h->d_D2T.p);
    });
    prof_launch(h, KC_COPYL, 0.0, lv.copyL.elems, [&] { launch_copy_L<T>(st, S, dev_list(h, lv.copyL), B); });
  }
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

gmrf_status check_status(gmrf_t h) {
  if (!(h->state & ST_FACTORED)) return GMRF_OK;
  int32_t s = INT_MAX, werr = 0;
  HIPCHK(h, hipMemcpyAsync(&s, h->d_status.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  if (h->d_sync.p)
    HIPCHK(h, hipMemcpyAsync(&werr, h->d_sync.p + h->sync_reset, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (werr != 0)
    return fail(h, GMRF_ERR_HIP, "a solve dependency wait exceeded its limit (results of that solve are invalid)");
  if (s != INT_MAX) {
    h->failed_index = (s >= 0 && s < h->n) ? h->sym.perm[s] : -1;
    return fail(h, GMRF_ERR_NOT_SPD, "matrix is not positive definite: non-positive pivot at original index " +
                                         std::to_string(h->failed_index));
  }
  h->failed_index = -1;
  return GMRF_OK;
}

// forward + backward (or backward only) solve of the FP64 pivot-order block xp (n x nrhs).
// skip (device, nullable, one right-hand side): when skip[0] == 0 the right-hand side is
// zero and the forest passes return at once.
template <typename T>
void run_solve(gmrf_t h, int nrhs, bool forward, const double* skip = nullptr) {
  const Symbolic& Y = h->sym;
  h->tsize = (int)sizeof(T);
  hipStream_t st = h->stream;
  const DevSym S = dev_sym(h);
  double* V[2] = {h->d_V0.p, h->d_V1.p};
  const T* Lp = (const T*)h->d_L.p;
  const T* D = (const T*)h->d_D.p;
  // several right-hand sides on a forest of small fronts (average supernode below 16,384
  // entries of L): one backward pass over the forest whose tasks take the columns in pairs,
  // each load of L serving both; large fronts keep the per-depth kernels, which read each
  // L block once for all columns
  const bool forest_multi = nrhs > 1 && !forward && Y.nnzL < (int64_t)16384 * Y.ns;
  if (nrhs == 1 || forest_multi) {
    // one launch per pass over the whole elimination forest
    int32_t* prog = h->d_sync.p;
    int32_t* kids = h->d_sync.p + Y.ns;
    int32_t* tick = h->d_sync.p + 2 * Y.ns + 2 * (Y.max_depth + 1);
    int32_t* err = h->d_sync.p + h->sync_reset;
    const ForestBufs G{h->d_sparent.p, h->d_fneed.p, kids, h->d_froff.p, h->d_fgptr.p, h->d_fgsrc.p,
                       h->d_fuoff.p, h->d_fU.p};
    double fb = 0.0;
    for (const Level& lv : h->levels) fb += lv.fbytes;
    if (forward) {
      launch_fill_i32(st, h->d_sync.p, h->sync_reset, 0);
      prof_launch(h, KC_FWD, 2.0 * fb, fb, [&] {
        launch_fwd_forest<T>(st, S, FusedTasks{h->d_ftasks.p, tick, prog, err, h->n_fgrp, h->d_fgrp.p},
                             G, Lp, D, h->d_xp.p, skip);
      });
    }
    launch_fill_i32(st, h->d_sync.p, h->sync_reset, 0);
    prof_launch(h, KC_BWD, 2.0 * fb * nrhs, fb, [&] {
      launch_bwd_forest<T>(st, S, FusedTasks{h->d_btasks.p, tick + 1, prog, err, h->n_bgrp, h->d_bgrp.p},
                           G, Lp, D, h->d_xp.p, nrhs, h->n, skip);
    });
    return;
  }
  if (forward) {
    for (int d = Y.max_depth; d >= 0; --d) {
      const Level& lv = h->levels[d];
      SolveBufs B{h->d_xp.p, V[d & 1], V[(d + 1) & 1], nrhs};
      prof_launch(h, KC_FWD, 0.0, 0.0, [&] {
        launch_fvec_init<T>(st, S, dev_list(h, lv.all), B);
        for (size_t c = 0; c < lv.fvec_ext.size(); ++c)
          launch_fvec_extend<T>(st, S, dev_list(h, lv.fvec_ext[c]), (int)c, B);
      });
      for (int t = 0; t < lv.nsteps2; ++t) {
        prof_launch(h, KC_FWD, nrhs * (lv.fblk[t].flops + lv.fout[t].flops), lv.fblk[t].elems + lv.fout[t].elems, [&] {
          launch_fwd_block<T>(st, S, dev_list(h, lv.fblk[t]), t, (const T*)h->d_D2.p, h->d_D2off.p, B);
          launch_fwd_outer<T>(st, S, dev_list(h, lv.fout[t]), t, Lp, B);
        });
      }
    }
  }
  for (int d = 0; d <= Y.max_depth; ++d) {
    const Level& lv = h->levels[d];
    SolveBufs B{h->d_xp.p, V[d & 1], V[(d + 1) & 1], nrhs};
    for (int t = 0; t < lv.nsteps2; ++t) {
      prof_launch(h, KC_BWD, nrhs * (lv.bpart[t].flops + lv.bblk[t].flops), lv.bpart[t].elems + lv.bblk[t].elems, [&] {
        launch_bwd_part<T>(st, S, dev_list(h, lv.bpart[t]), t, Lp, B, h->d_bpart.p);
        launch_bwd_block<T>(st, S, dev_list(h, lv.bblk[t]), dev_list(h, lv.bpart[t]), t, (const T*)h->d_D2T.p,
                            h->d_D2off.p, B, h->d_bpart.p);
      });
    }
  }
}

gmrf_status alloc_solve(gmrf_t h, int nrhs) {
  const Symbolic& Y = h->sym;
  HIPCHK(h, h->d_V0.alloc((size_t)std::max<int64_t>(Y.Vsize[0], 1) * nrhs));
  HIPCHK(h, h->d_V1.alloc((size_t)std::max<int64_t>(Y.Vsize[1], 1) * nrhs));
  HIPCHK(h, h->d_xp.alloc((size_t)h->n * nrhs));
  HIPCHK(h, h->d_w.alloc(h->n));
  HIPCHK(h, h->d_r.alloc(h->n));
  HIPCHK(h, h->d_red.alloc(1024));
  HIPCHK(h, h->d_norm.alloc(4));
  HIPCHK(h, h->d_mu_post.alloc(h->n));
  HIPCHK(h, h->d_bpart.alloc((size_t)std::max<int64_t>(h->bpart_max, 1) * kNB2 * 16));
  return GMRF_OK;
}

template <typename T>
gmrf_status run_selinv(gmrf_t h, double* var, double* sigq) {
  const Symbolic& Y = h->sym;
  hipStream_t st = h->stream;
  const DevSym S = dev_sym(h);
  h->tsize = (int)sizeof(T);
  int64_t ysz = std::max<int64_t>(std::max(Y.Vsize[0], Y.Vsize[1]), 1) * kNB2;
  HIPCHK(h, h->d_Y.alloc((size_t)ysz * sizeof(T)));
  HIPCHK(h, h->d_part.alloc((size_t)std::max<int64_t>(h->part_max, 1) * kNB * kNB * sizeof(T)));
  {
    const size_t gp = std::is_same<T, float>::value ? (size_t)std::max<int64_t>(h->gpart3_max, 1) * 256 * 128
                                                     : (size_t)std::max<int64_t>(h->gpart_max, 1) * kBigTile * kBigTile;
    HIPCHK(h, h->d_gpart.alloc(gp * sizeof(T)));
  }
  T* W[2] = {(T*)h->d_W0.p, (T*)h->d_W1.p};
  T* D2 = (T*)h->d_D2.p;
  for (int d = 0; d <= Y.max_depth; ++d) {
    const Level& lv = h->levels[d];
    SelBufs<T> B;
    B.L = (const T*)h->d_L.p;
    B.D = (const T*)h->d_D.p;
    B.Scur = W[d & 1];
    B.Spar = W[(d + 1) & 1];   // parent depth d-1 has the other parity
    B.Y = (T*)h->d_Y.p;
    B.part = (T*)h->d_part.p;
    B.gpart = (T*)h->d_gpart.p;
    prof_launch(h, KC_SEL_GATHER, 0.0, lv.sgather.elems,
                [&] { launch_sel_gather<T>(st, S, dev_list(h, lv.sgather), h->d_sparent.p, B); });
    for (int t = 0; t < lv.nsteps2; ++t) {
      prof_launch(h, KC_SEL_Y, lv.sY2[t].flops, lv.sY2[t].elems,
                  [&] { launch_sel_Y2<T>(st, S, dev_list(h, lv.sY2[t]), t, B, h->d_D2off.p, (const T*)h->d_D2T.p); });
      const bool f32 = std::is_same<T, float>::value;
      const HostList& G = f32 ? lv.sgemm4[t] : lv.sgemm2[t];
      const HostList& R = f32 ? lv.sgred4[t] : lv.sgred[t];
      if (G.total > 0)
        prof_launch(h, KC_SEL_GEMM, G.flops, G.elems, [&] {
          if constexpr (std::is_same<T, float>::value) launch_sel_gemm4(st, S, dev_list(h, G), t, B);
          else launch_sel_gemm2<T>(st, S, dev_list(h, G), t, B);
        });
      if (R.total > 0)
        prof_launch(h, KC_SEL_RED, 0.0, R.elems,
                    [&] { launch_sel_gemm_reduce<T>(st, S, dev_list(h, R), t, B); });
      if (f32 && lv.sgemm2s[t].total > 0)
        prof_launch(h, KC_SEL_GEMM_S, lv.sgemm2s[t].flops, lv.sgemm2s[t].elems,
                    [&] { launch_sel_gemm2<T>(st, S, dev_list(h, lv.sgemm2s[t]), t, B); });
      prof_launch(h, KC_SEL_DIAG, lv.spart2[t].flops + lv.sfin2[t].flops, lv.spart2[t].elems + lv.sfin2[t].elems, [&] {
        launch_sel_part2<T>(st, S, dev_list(h, lv.spart2[t]), t, B);
        launch_sel_fin2<T>(st, S, dev_list(h, lv.sfin2[t]), dev_list(h, lv.spart2[t]), t, B, h->d_D2off.p, D2);
      });
    }
    prof_launch(h, KC_SEL_OUT, 0.0, 0.0, [&] {
      launch_sel_extract<T>(st, S, dev_list(h, lv.all), B, h->d_scale.p, var);
      if (sigq)
        launch_sel_pattern<T>(st, lv.map_end - lv.map_begin, h->d_map_e.p + lv.map_begin,
                              h->d_map_off.p + lv.map_begin, h->d_qrow.p, h->d_qci.p, h->d_scale.p, B.Scur,
                              sigq);
    });
  }
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

gmrf_status assemble_device(gmrf_t h) {
  hipStream_t st = h->stream;
  launch_assemble_qpost(st, h->nnzq, h->d_qval.p, h->d_cptr.p, h->d_cpair.p, h->d_arow.p, h->d_aval.p,
                        h->d_qeps.p, h->d_qpost.p);
  if (h->m > 0) {
    launch_obs_residual(st, h->m, h->d_arp.p, h->d_aci.p, h->d_aval.p, h->d_qeps.p, h->d_y.p,
                        h->has_b ? h->d_b.p : nullptr, h->has_mu ? h->d_mu.p : nullptr, h->d_rvec.p);
    launch_at_times(st, h->n, h->d_atp.p, h->d_ati.p, h->d_arow.p, h->d_aval.p, h->d_rvec.p, h->d_h.p);
  } else {
    launch_fill_f64(st, h->d_h.p, h->n, 0.0);
  }
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

// ------------------------------------------------------------------ Gauss-Newton driver
constexpr int kGNRec = 6;   // doubles per Gauss-Newton iteration record

struct GNArgs {
  int kind;                  // 0: Burgers (Galerkin implicit Euler); 1: pointwise power
  int64_t nx, nt;            // Burgers
  double dt, nu;
  const double* mass;
  const double* s3;
  const double* lin;         // pointwise: linear part of A (A's pattern), unknown of the
  const int32_t* nl_col;     // nonlinear term per row (-1: none), its coefficient, power
  const double* nl_coef;
  int power;
  double* u;
  int refine;
  double tol;
};

// linearise the residual at u into A's values and b (Sec. 3.3)
void gn_linearize(gmrf_t h, const GNArgs& a) {
  if (a.kind == 0)
    launch_burgers_linearize(h->stream, a.nx, a.nt, a.dt, a.nu, a.mass, a.s3, a.u, h->d_arp.p, h->d_aval.p,
                             h->d_b.p);
  else
    launch_pw_linearize(h->stream, h->m, h->d_arp.p, h->d_aci.p, a.lin, a.nl_col, a.nl_coef, a.power, a.u,
                        h->d_aval.p, h->d_b.p);
}

// solve Q_post x = h on device only (no host synchronisation, capturable): one solve
// plus at most `refine` corrections with FP64 residuals.  A device gate stops the
// corrections once ||h - Q_post x|| <= tol ||h|| (the remaining ones have a zero
// right-hand side, their forest passes return at once and they add nothing); rec[0]
// receives the final relative residual and rec[1] the number of corrections applied.
template <typename T>
void device_solve(gmrf_t h, double* x, int refine, double tol, double* rec) {
  hipStream_t st = h->stream;
  const int64_t n = h->n;
  double* gate = h->d_gn_sel.p + 1;   // gate[0]: apply the next correction; gate[1]: count
  launch_norm2(st, n, h->d_h.p, h->d_red.p, h->d_norm.p + 0);
  launch_fill_f64(st, gate, 2, 0.0);
  launch_permute_in(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_h.p, n, h->d_xp.p);
  run_solve<T>(h, 1, true);
  launch_permute_out(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_xp.p, nullptr, 0, x, n, 0);
  for (int it = 0; it < refine; ++it) {
    launch_resid(st, n, h->d_qrp.p, h->d_qci.p, h->d_qpost.p, h->d_h.p, x, h->d_r.p);
    launch_norm2(st, n, h->d_r.p, h->d_red.p, h->d_norm.p + 1);
    launch_refine_gate(st, h->d_norm.p, tol, gate, nullptr, 0);
    launch_permute_in(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_r.p, n, h->d_xp.p, gate);
    run_solve<T>(h, 1, true, gate);
    launch_permute_out(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_xp.p, nullptr, 0, x, n, 1);
  }
  launch_resid(st, n, h->d_qrp.p, h->d_qci.p, h->d_qpost.p, h->d_h.p, x, h->d_r.p);
  launch_norm2(st, n, h->d_r.p, h->d_red.p, h->d_norm.p + 1);
  launch_refine_gate(st, h->d_norm.p, tol, gate, rec, 1);
}

// one Gauss-Newton iteration, fully asynchronous (capturable): linearise at u, assemble
// H = Q + J^T Q_eps J and the right-hand side, factor (same pattern, reused analysis),
// solve for the linearised posterior mean x, direction d = x - u, batched backtracking
// line search on the device, u += alpha d.  The iteration record lands in
// d_gn_rec[0..5] (objective, step, decrement, slope, refinement residual, corrections).
template <typename T>
gmrf_status gn_body(gmrf_t h, const GNArgs& a) {
  hipStream_t st = h->stream;
  const int64_t n = h->n;
  gn_linearize(h, a);
  gmrf_status rc = assemble_device(h);
  if (rc != GMRF_OK) return rc;
  rc = run_factor<T>(h);
  if (rc != GMRF_OK) return rc;
  device_solve<T>(h, h->d_gn_x.p, a.refine, a.tol, h->d_gn_rec.p + 4);
  launch_gn_direction(st, n, h->d_gn_x.p, a.u, h->d_gn_d.p);
  launch_spmv(st, n, h->d_qrp.p, h->d_qci.p, h->d_qval.p, a.u, h->d_gn_tmp.p);
  launch_dot(st, n, a.u, h->d_gn_tmp.p, h->d_red.p, h->d_gn_quad.p + 0);
  launch_dot(st, n, h->d_gn_d.p, h->d_gn_tmp.p, h->d_red.p, h->d_gn_quad.p + 1);
  launch_spmv(st, n, h->d_qrp.p, h->d_qci.p, h->d_qval.p, h->d_gn_d.p, h->d_gn_tmp.p);
  launch_dot(st, n, h->d_gn_d.p, h->d_gn_tmp.p, h->d_red.p, h->d_gn_quad.p + 2);
  if (a.kind == 0)
    launch_gn_linesearch(st, a.nx, a.nt, a.dt, a.nu, a.mass, a.s3, a.u, h->d_gn_d.p, h->d_y.p, h->d_qeps.p,
                         h->d_arp.p, h->d_aci.p, h->d_aval.p, h->d_gn_part.p, h->d_gn_quad.p, h->d_gn_sel.p,
                         h->d_gn_rec.p);
  else
    launch_pw_linesearch(st, h->m, h->d_arp.p, h->d_aci.p, a.lin, a.nl_col, a.nl_coef, a.power, a.u, h->d_gn_d.p,
                         h->d_y.p, h->d_qeps.p, h->d_aval.p, h->d_gn_part.p, h->d_gn_quad.p, h->d_gn_sel.p,
                         h->d_gn_rec.p);
  launch_gn_update(st, n, h->d_gn_sel.p, h->d_gn_d.p, a.u);
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

// Gauss-Newton iterations on the device (Sec. 3.3) for either residual model: iteration 0
// eager, the later ones replaying one hipGraph captured by this call; then the Laplace
// approximation at the final iterate (relinearised and refactored).
gmrf_status gn_run(gmrf_t h, const GNArgs& a, int iters, int precision, int use_graph, double decrement_tol,
                   double* rec_out) {
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, GMRF_ERR_HIP, "hipSetDevice failed");
  hipStream_t user = h->stream;
  if (!h->gn_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->gn_stream, hipStreamNonBlocking));
  HIPCHK(h, user ? hipStreamSynchronize(user) : hipDeviceSynchronize());
  h->stream = h->gn_stream;
  // The graph captured by this call holds this call's pointers and sizes (u, mass, the
  // library's current buffers), so it lives only for this call: every exit drains the
  // stream and destroys it.
  struct Restore {
    gmrf_t h;
    hipStream_t s;
    ~Restore() {
      if (h->gn_exec) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipGraphExecDestroy(h->gn_exec);
        h->gn_exec = nullptr;
      }
      h->stream = s;
    }
  } restore{h, user};
  const bool prof = h->prof;
  h->prof = false;
  HIPCHK(h, h->d_gn_x.alloc(h->n));
  HIPCHK(h, h->d_gn_d.alloc(h->n));
  HIPCHK(h, h->d_gn_tmp.alloc(h->n));
  HIPCHK(h, h->d_gn_part.alloc(10 * 256));
  HIPCHK(h, h->d_gn_quad.alloc(4));
  HIPCHK(h, h->d_gn_sel.alloc(3));
  HIPCHK(h, h->d_gn_rec.alloc(kGNRec));
  gmrf_status rc = alloc_solve(h, 1);
  if (rc != GMRF_OK) return rc;
  rc = precision == GMRF_FP64 ? alloc_numeric<double>(h) : alloc_numeric<float>(h);
  if (rc != GMRF_OK) return rc;
  h->has_b = true;
  std::vector<double> rec(kGNRec * (size_t)iters, 0.0);
  auto body = [&]() { return precision == GMRF_FP64 ? gn_body<double>(h, a) : gn_body<float>(h, a); };
  HIPCHK(h, hipEventRecord(h->ev[0], h->stream));
  for (int it = 0; it < iters; ++it) {
    const bool graph = use_graph && it > 0;
    if (graph && !h->gn_exec) {
      hipGraph_t g = nullptr;
      HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      rc = body();
      hipError_t ce = hipStreamEndCapture(h->stream, &g);
      if (rc != GMRF_OK) { if (g) (void)hipGraphDestroy(g); return rc; }
      HIPCHK(h, ce);
      hipError_t ie = hipGraphInstantiate(&h->gn_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPCHK(h, ie);
    }
    if (graph) {
      HIPCHK(h, hipGraphLaunch(h->gn_exec, h->stream));
    } else {
      rc = body();
      if (rc != GMRF_OK) return rc;
    }
    HIPCHK(h, hipMemcpyAsync(rec.data() + kGNRec * it, h->d_gn_rec.p, kGNRec * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
    if (decrement_tol > 0.0) {
      // stopping rule: the Newton decrement lambda^2 / 2 = -grad^T d / 2 of this
      // iteration's direction below decrement_tol, or no step taken (the objective cannot
      // decrease any more); the records of the iterations not run are NaN
      HIPCHK(h, hipStreamSynchronize(h->stream));
      const double* r = rec.data() + kGNRec * it;
      if ((r[2] >= 0.0 && 0.5 * r[2] < decrement_tol) || r[1] == 0.0) {
        std::fill(rec.begin() + kGNRec * (it + 1), rec.end(), std::numeric_limits<double>::quiet_NaN());
        break;
      }
    }
  }
  HIPCHK(h, hipEventRecord(h->ev[1], h->stream));
  // Laplace approximation at the final iterate (Sec. 3.3): relinearise and refactor so that
  // logdet / sample / selinv describe N(u*, (Q + J*^T Q_eps J*)^-1)
  gn_linearize(h, a);
  rc = assemble_device(h);
  if (rc != GMRF_OK) return rc;
  rc = precision == GMRF_FP64 ? run_factor<double>(h) : run_factor<float>(h);
  if (rc != GMRF_OK) return rc;
  HIPCHK(h, copy_d2d(h->d_mu_post.p, a.u, h->n * sizeof(double), h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->ev_factor = false;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, h->ev[0], h->ev[1]) == hipSuccess) h->phase_ms[0] = ms;
  h->prof = prof;
  h->prec = precision;
  h->state |= ST_FACTORED | ST_SOLVED;
  if (rec_out) std::memcpy(rec_out, rec.data(), rec.size() * sizeof(double));
  return check_status(h);
}


// Preconditioned CG for Q_post x = b on the device (FP64 vectors, fixed-order dots); the
// preconditioner is the diagonal of Q_post (precond 0) or the context's factor (1: one
// forward and one backward solve per iteration).  The relative residual is checked on the
// host after every iteration.  Returns the iterations and the final relative residual.
template <typename T>
void pcg_solve(gmrf_t h, const double* b, double* x, bool warm, int precond, int maxit, double tol, int* its,
               double* rel) {
  hipStream_t st = h->stream;
  const int64_t n = h->n;
  double* r = h->d_cg.p;
  double* z = r + n;
  double* p = z + n;
  double* q = p + n;
  double* sc = q + n;           // (r^T z, p^T q, new r^T z, ||r||, ||b||)
  auto precondition = [&](const double* in, double* out) {
    if (precond == 0) {
      launch_jacobi(st, n, h->d_qdiag.p, h->d_qpost.p, in, out);
    } else {
      launch_permute_in(st, n, 1, h->d_perm.p, h->d_scale.p, in, n, h->d_xp.p);
      run_solve<T>(h, 1, true);
      launch_permute_out(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_xp.p, nullptr, 0, out, n, 0);
    }
  };
  if (!warm) launch_fill_f64(st, x, n, 0.0);
  launch_resid(st, n, h->d_qrp.p, h->d_qci.p, h->d_qpost.p, b, x, r);   // r = b - Q x
  launch_norm2(st, n, b, h->d_red.p, sc + 4);
  if (precond == 0) {
    // diagonal preconditioner: five launches per iteration (sc[0], sc[1]: r^T z of the
    // current and next iteration, sc[2]: p^T q, sc[5]: ||r||^2); the residual norm is read on
    // the host every kCgCheck iterations (and at maxit), so up to kCgCheck - 1 iterations
    // may run past the one that first met the tolerance
    constexpr int kCgCheck = 8;
    launch_jacobi(st, n, h->d_qdiag.p, h->d_qpost.p, r, z);
    launch_copy_f64(st, n, z, p);
    launch_dot(st, n, r, z, h->d_red.p, sc + 0);
    launch_norm2(st, n, r, h->d_red.p, sc + 3);
    double hs[2] = {0.0, 0.0};
    int it = 0, cur = 0;
    double rr = 0.0;
    while (true) {
      if (it % kCgCheck == 0 || it >= maxit) {
        if (it > 0) launch_partial_norm(st, h->d_cgpart.p, sc + 3);
        if (hipMemcpyAsync(hs, sc + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) break;
        if (hipStreamSynchronize(st) != hipSuccess) break;
        rr = hs[0] / (hs[1] > 0.0 ? hs[1] : 1.0);
        if (rr <= tol || it >= maxit || !std::isfinite(rr)) break;
      }
      launch_cg_iteration(st, n, h->d_qrp.p, h->d_qci.p, h->d_qpost.p, h->d_qdiag.p, sc, cur, x, r, z, p, q,
                          h->d_cgpart.p);
      cur ^= 1;
      ++it;
    }
    *its = it;
    *rel = rr;
    return;
  }
  precondition(r, z);
  launch_copy_f64(st, n, z, p);
  launch_dot(st, n, r, z, h->d_red.p, sc + 0);
  double hs[2] = {0.0, 0.0};
  int it = 0;
  double rr = 0.0;
  while (true) {
    launch_norm2(st, n, r, h->d_red.p, sc + 3);
    if (hipMemcpyAsync(hs, sc + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess) break;
    if (hipStreamSynchronize(st) != hipSuccess) break;
    rr = hs[0] / (hs[1] > 0.0 ? hs[1] : 1.0);
    if (rr <= tol || it >= maxit || !std::isfinite(rr)) break;
    launch_spmv(st, n, h->d_qrp.p, h->d_qci.p, h->d_qpost.p, p, q);
    launch_dot(st, n, p, q, h->d_red.p, sc + 1);
    launch_cg_xr(st, n, sc, p, q, x, r);
    precondition(r, z);
    launch_dot(st, n, r, z, h->d_red.p, sc + 2);
    launch_cg_p(st, n, sc, z, p);
    ++it;
  }
  *its = it;
  *rel = rr;
}

gmrf_status pcg_prepare(gmrf_t h, int precond) {
  if (!(h->state & ST_ASSEMBLED) || !(h->state & ST_ANALYZED))
    return fail(h, GMRF_ERR_STATE, "conjugate gradients need gmrf_assemble and gmrf_analyze");
  if (precond != 0 && precond != 1) return fail(h, GMRF_ERR_ARG, "precond must be 0 (diagonal) or 1 (factor)");
  if (precond == 1) {
    if (!(h->state & ST_FACTORED)) return fail(h, GMRF_ERR_STATE, "precond 1 needs gmrf_factor");
    gmrf_status rc = check_status(h);
    if (rc != GMRF_OK) return rc;
  }
  gmrf_status rc = alloc_solve(h, 1);
  if (rc != GMRF_OK) return rc;
  HIPCHK(h, h->d_cg.alloc((size_t)(4 * h->n + 8)));
  HIPCHK(h, h->d_cgpart.alloc((size_t)kCgPartials));
  return GMRF_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

gmrf_status gmrf_create(gmrf_t* out, int device, void* hip_stream) {
  if (!out) return GMRF_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GMRF_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return GMRF_ERR_HIP;
  gmrf_t h = new gmrf_ctx();
  h->device = device;
  h->stream = (hipStream_t)hip_stream;
  for (auto& e : h->ev) {
    if (hipEventCreate(&e) != hipSuccess) { delete h; return GMRF_ERR_HIP; }
  }
  // device address of the no-allocation workspace, once per device (this device is current)
  if (device < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        for (auto& e : h->ev) (void)hipEventDestroy(e);
        delete h;
        return GMRF_ERR_HIP;
      }
      g_scratch_dev[device] = ptr;
    }
  }
  *out = h;
  return GMRF_OK;
}

gmrf_status gmrf_destroy(gmrf_t h) {
  if (!h) return GMRF_OK;
  (void)hipSetDevice(h->device);
  (void)sel_sync(h);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  if (h->sel_stream) (void)hipStreamDestroy(h->sel_stream);
  if (h->ev_sel_start) (void)hipEventDestroy(h->ev_sel_start);
  if (h->ev_sel_done) (void)hipEventDestroy(h->ev_sel_done);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : h->evpool)
    if (e) (void)hipEventDestroy(e);
  if (h->gn_exec) (void)hipGraphExecDestroy(h->gn_exec);
  if (h->gn_stream) (void)hipStreamDestroy(h->gn_stream);
  delete h;
  return GMRF_OK;
}

const char* gmrf_last_error(gmrf_t h) {
  if (!h) return "null handle";
  return h->err.c_str();
}

gmrf_status gmrf_assemble(gmrf_t h, int64_t n, const int64_t* q_rowptr, const int32_t* q_col,
                          const double* q_val, int64_t m, const int64_t* a_rowptr, const int32_t* a_col,
                          const double* a_val, const double* q_eps, const double* y, const double* b,
                          const double* mu_prior, int64_t n_blocks, const int64_t* block_ptr) {
  if (!h) return GMRF_ERR_ARG;
  HIPCHK(h, sel_sync(h));
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, GMRF_ERR_HIP, "hipSetDevice failed");
  hipStream_t st = h->stream;
  if (n <= 0 || m < 0 || !q_rowptr || !q_col || !q_val) return fail(h, GMRF_ERR_ARG, "bad sizes or null Q");
  if (m > 0 && (!a_rowptr || !a_col || !a_val || !q_eps || !y)) return fail(h, GMRF_ERR_ARG, "null A arrays");
  int64_t nnzq = 0, nnza = 0;
  HIPCHK(h, hipMemcpy(&nnzq, q_rowptr + n, sizeof(int64_t), hipMemcpyDeviceToHost));
  if (m > 0) HIPCHK(h, hipMemcpy(&nnza, a_rowptr + m, sizeof(int64_t), hipMemcpyDeviceToHost));
  const bool first = !(h->state & ST_ASSEMBLED);
  if (!first && (n != h->n || m != h->m || nnzq != h->nnzq || nnza != h->nnza))
    return fail(h, GMRF_ERR_PATTERN, "pattern differs from the first gmrf_assemble of this context");
  if (first) {
    if (nnzq <= 0 || nnzq >= ((int64_t)1 << 40)) return fail(h, GMRF_ERR_ARG, "bad nnz(Q)");
    if (nnza >= ((int64_t)1 << 31)) return fail(h, GMRF_ERR_ARG, "nnz(A) must be below 2^31");
    h->n = n; h->m = m; h->nnzq = nnzq; h->nnza = nnza;
    HIPCHK(h, download(h->qrp, q_rowptr, (size_t)n + 1, st));
    HIPCHK(h, download(h->qci, q_col, (size_t)nnzq, st));
    if (m > 0) {
      HIPCHK(h, download(h->arp, a_rowptr, (size_t)m + 1, st));
      HIPCHK(h, download(h->aci, a_col, (size_t)nnza, st));
    } else {
      h->arp.assign(1, 0);
      h->aci.clear();
    }
    std::string e = check_csr(n, n, h->qrp, h->qci, "Q");
    if (e.empty() && m > 0) e = check_csr(m, n, h->arp, h->aci, "A");
    if (!e.empty()) { h->state = 0; return fail(h, GMRF_ERR_ARG, e); }
    // diagonal, symmetry
    std::vector<int64_t> qdiag(n);
    std::vector<int32_t> qrow(nnzq);
    for (int64_t r = 0; r < n; ++r) {
      int64_t dpos = find_entry(h->qrp, h->qci, r, (int32_t)r);
      if (dpos < 0) { h->state = 0; return fail(h, GMRF_ERR_ARG, "Q lacks diagonal entry " + std::to_string(r)); }
      qdiag[r] = dpos;
      for (int64_t q = h->qrp[r]; q < h->qrp[r + 1]; ++q) {
        qrow[q] = (int32_t)r;
        if (find_entry(h->qrp, h->qci, h->qci[q], (int32_t)r) < 0) {
          h->state = 0;
          return fail(h, GMRF_ERR_ARG, "pattern of Q is not symmetric");
        }
      }
    }
    // A row index, A^T (CSC) and the contribution list of A^T Q_eps A on Q's pattern
    std::vector<int32_t> arow(nnza);
    for (int64_t r = 0; r < m; ++r)
      for (int64_t q = h->arp[r]; q < h->arp[r + 1]; ++q) arow[q] = (int32_t)r;
    std::vector<int64_t> atp(n + 1, 0);
    for (int64_t q = 0; q < nnza; ++q) atp[h->aci[q] + 1]++;
    for (int64_t i = 0; i < n; ++i) atp[i + 1] += atp[i];
    std::vector<int32_t> ati(nnza);
    {
      std::vector<int64_t> fill(atp.begin(), atp.end() - 1);
      for (int64_t q = 0; q < nnza; ++q) ati[fill[h->aci[q]]++] = (int32_t)q;
    }
    std::vector<int64_t> cptr(nnzq + 1, 0);
    for (int64_t r = 0; r < m; ++r) {
      for (int64_t a1 = h->arp[r]; a1 < h->arp[r + 1]; ++a1) {
        for (int64_t a2 = h->arp[r]; a2 < h->arp[r + 1]; ++a2) {
          int64_t e2 = find_entry(h->qrp, h->qci, h->aci[a1], h->aci[a2]);
          if (e2 < 0) {
            h->state = 0;
            return fail(h, GMRF_ERR_ARG, "A^T Q_eps A has an entry outside the pattern of Q");
          }
          cptr[e2 + 1]++;
        }
      }
    }
    for (int64_t e2 = 0; e2 < nnzq; ++e2) cptr[e2 + 1] += cptr[e2];
    std::vector<int32_t> cpair(2 * (size_t)cptr[nnzq]);
    {
      std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
      for (int64_t r = 0; r < m; ++r)
        for (int64_t a1 = h->arp[r]; a1 < h->arp[r + 1]; ++a1)
          for (int64_t a2 = h->arp[r]; a2 < h->arp[r + 1]; ++a2) {
            int64_t e2 = find_entry(h->qrp, h->qci, h->aci[a1], h->aci[a2]);
            int64_t q = fill[e2]++;
            cpair[2 * q] = (int32_t)a1;
            cpair[2 * q + 1] = (int32_t)a2;
          }
    }
    HIPCHK(h, upload(h->d_qrp, h->qrp, st));
    HIPCHK(h, upload(h->d_qci, h->qci, st));
    HIPCHK(h, upload(h->d_qrow, qrow, st));
    HIPCHK(h, upload(h->d_qdiag, qdiag, st));
    HIPCHK(h, upload(h->d_arp, h->arp, st));
    HIPCHK(h, upload(h->d_aci, h->aci, st));
    HIPCHK(h, upload(h->d_arow, arow, st));
    HIPCHK(h, upload(h->d_atp, atp, st));
    HIPCHK(h, upload(h->d_ati, ati, st));
    HIPCHK(h, upload(h->d_cptr, cptr, st));
    HIPCHK(h, upload(h->d_cpair, cpair, st));
    HIPCHK(h, h->d_qval.alloc(nnzq));
    HIPCHK(h, h->d_aval.alloc(std::max<int64_t>(nnza, 1)));
    HIPCHK(h, h->d_qeps.alloc(std::max<int64_t>(m, 1)));
    HIPCHK(h, h->d_y.alloc(std::max<int64_t>(m, 1)));
    HIPCHK(h, h->d_b.alloc(std::max<int64_t>(m, 1)));
    HIPCHK(h, h->d_mu.alloc(n));
    HIPCHK(h, h->d_qpost.alloc(nnzq));
    HIPCHK(h, h->d_h.alloc(n));
    HIPCHK(h, h->d_rvec.alloc(std::max<int64_t>(m, 1)));
    // blocks
    h->nblocks = 1;
    h->block_ptr.assign({0, n});
    if (n_blocks > 0 && block_ptr) {
      if (block_ptr[0] != 0 || block_ptr[n_blocks] != n) return fail(h, GMRF_ERR_ARG, "block_ptr must span 0..n");
      for (int64_t q = 0; q < n_blocks; ++q)
        if (block_ptr[q + 1] < block_ptr[q]) return fail(h, GMRF_ERR_ARG, "block_ptr decreases");
      h->nblocks = n_blocks;
      h->block_ptr.assign(block_ptr, block_ptr + n_blocks + 1);
    }
  }
  HIPCHK(h, copy_d2d(h->d_qval.p, q_val, nnzq * sizeof(double), st));
  if (m > 0) {
    HIPCHK(h, copy_d2d(h->d_aval.p, a_val, nnza * sizeof(double), st));
    HIPCHK(h, copy_d2d(h->d_qeps.p, q_eps, m * sizeof(double), st));
    HIPCHK(h, copy_d2d(h->d_y.p, y, m * sizeof(double), st));
  }
  h->has_b = b != nullptr;
  h->has_mu = mu_prior != nullptr;
  if (b && m > 0) HIPCHK(h, copy_d2d(h->d_b.p, b, m * sizeof(double), st));
  if (mu_prior) HIPCHK(h, copy_d2d(h->d_mu.p, mu_prior, n * sizeof(double), st));
  gmrf_status rc = assemble_device(h);
  if (rc != GMRF_OK) return rc;
  h->state |= ST_ASSEMBLED;
  h->state &= ~(ST_FACTORED | ST_SOLVED);
  return GMRF_OK;
}

gmrf_status gmrf_update_values(gmrf_t h, const double* q_val, const double* a_val, const double* q_eps,
                               const double* y, const double* b) {
  if (!h) return GMRF_ERR_ARG;
  HIPCHK(h, sel_sync(h));
  if (!(h->state & ST_ASSEMBLED)) return fail(h, GMRF_ERR_STATE, "gmrf_update_values before gmrf_assemble");
  hipStream_t st = h->stream;
  if (q_val) HIPCHK(h, copy_d2d(h->d_qval.p, q_val, h->nnzq * sizeof(double), st));
  if (h->m > 0) {
    if (a_val) HIPCHK(h, copy_d2d(h->d_aval.p, a_val, h->nnza * sizeof(double), st));
    if (q_eps) HIPCHK(h, copy_d2d(h->d_qeps.p, q_eps, h->m * sizeof(double), st));
    if (y) HIPCHK(h, copy_d2d(h->d_y.p, y, h->m * sizeof(double), st));
    if (b) { HIPCHK(h, copy_d2d(h->d_b.p, b, h->m * sizeof(double), st)); h->has_b = true; }
  }
  gmrf_status rc = assemble_device(h);
  if (rc != GMRF_OK) return rc;
  h->state &= ~(ST_FACTORED | ST_SOLVED);
  return GMRF_OK;
}

static void fill_opts(const gmrf_options* o, AnalyzeOptions& opt) {
  opt = AnalyzeOptions();
  if (!o) return;
  if (o->leaf_size > 0) opt.leaf_size = o->leaf_size;
  if (o->relax_small > 0) opt.relax_small = o->relax_small;
  if (o->relax_mid > 0) opt.relax_mid = o->relax_mid;
  if (o->relax_big > 0) opt.relax_big = o->relax_big;
}

gmrf_status gmrf_analyze(gmrf_t h, const double* coords, int dim, const gmrf_options* opts) {
  if (!h) return GMRF_ERR_ARG;
  HIPCHK(h, sel_sync(h));
  if (!(h->state & ST_ASSEMBLED)) return fail(h, GMRF_ERR_STATE, "gmrf_analyze before gmrf_assemble");
  if (coords && (dim < 1 || dim > 3)) return fail(h, GMRF_ERR_ARG, "dim must be 1..3");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, GMRF_ERR_HIP, "hipSetDevice failed");
  fill_opts(opts, h->opt);
  h->opt.nb = kNB;
  std::string e = analyze(h->n, h->qrp.data(), h->qci.data(), coords, coords ? dim : 0, h->opt, h->sym);
  if (!e.empty()) return fail(h, GMRF_ERR_ARG, e);
  gmrf_status rc = build_plan(h);
  if (rc != GMRF_OK) return rc;
  h->state = (h->state & ST_ASSEMBLED) | ST_ANALYZED;
  h->prec = -1;
  return GMRF_OK;
}

gmrf_status gmrf_factor(gmrf_t h, gmrf_precision p) {
  if (!h) return GMRF_ERR_ARG;
  HIPCHK(h, sel_sync(h));
  if (!(h->state & ST_ANALYZED)) return fail(h, GMRF_ERR_STATE, "gmrf_factor before gmrf_analyze");
  if (p != GMRF_FP64 && p != GMRF_FP32_REFINE) return fail(h, GMRF_ERR_ARG, "unknown precision");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, GMRF_ERR_HIP, "hipSetDevice failed");
  HIPCHK(h, hipEventRecord(h->ev[0], h->stream));
  gmrf_status rc = p == GMRF_FP64 ? run_factor<double>(h) : run_factor<float>(h);
  if (rc != GMRF_OK) return rc;
  HIPCHK(h, hipEventRecord(h->ev[1], h->stream));
  h->ev_factor = true;
  h->prec = (int)p;
  h->state |= ST_FACTORED;
  h->state &= ~ST_SOLVED;
  return GMRF_OK;
}

gmrf_status gmrf_logdet(gmrf_t h, double* out) {
  if (!h || !out) return fail(h, GMRF_ERR_ARG, "null argument");
  if (!(h->state & ST_FACTORED)) return fail(h, GMRF_ERR_STATE, "gmrf_logdet before gmrf_factor");
  gmrf_status rc = check_status(h);
  if (rc != GMRF_OK) return rc;
  HIPCHK(h, h->d_ld.alloc(h->nblocks * 65));
  prof_launch(h, KC_LOGDET, 0.0, 0.0, [&] {
    launch_logdet(h->stream, h->nblocks, h->d_bptr.p, h->d_bpiv.p, h->d_perm.p, h->d_piv.p, h->d_sexp.p,
                  h->d_ld.p + h->nblocks, h->d_ld.p);
  });
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(out, h->d_ld.p, h->nblocks * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return GMRF_OK;
}

gmrf_status gmrf_logdet_noalloc(gmrf_t h, double* out_dev) {
  if (!h || !out_dev) return fail(h, GMRF_ERR_ARG, "null argument");
  if (h->nblocks > kNoAllocMaxBlocks)
    return fail(h, GMRF_ERR_ARG, "gmrf_logdet_noalloc: " + std::to_string(h->nblocks) +
                                     " blocks exceed its workspace of " + std::to_string(kNoAllocMaxBlocks));
  if (!(h->state & ST_FACTORED)) return fail(h, GMRF_ERR_STATE, "gmrf_logdet_noalloc before gmrf_factor");
  void* ws = h->device < kMaxDevices ? g_scratch_dev[h->device] : nullptr;
  if (!ws) return fail(h, GMRF_ERR_STATE, "no-allocation workspace unavailable on this device");
  // every partial is written before it is read: nothing to clear; no profiler events
  launch_logdet(h->stream, h->nblocks, h->d_bptr.p, h->d_bpiv.p, h->d_perm.p, h->d_piv.p, h->d_sexp.p,
                (double*)ws, out_dev);
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

gmrf_status gmrf_solve(gmrf_t h, double* mu_out, int max_refine, double tol, int* iters_out, double* resid_out) {
  if (!h || !mu_out) return fail(h, GMRF_ERR_ARG, "null argument");
  if (!(h->state & ST_FACTORED)) return fail(h, GMRF_ERR_STATE, "gmrf_solve before gmrf_factor");
  gmrf_status rc = check_status(h);
  if (rc != GMRF_OK) return rc;
  rc = alloc_solve(h, 1);
  if (rc != GMRF_OK) return rc;
  hipStream_t st = h->stream;
  const int64_t n = h->n;
  const bool f32 = h->prec == GMRF_FP32_REFINE;
  HIPCHK(h, hipEventRecord(h->ev[2], st));
  // w = Q_post^-1 h:  w = S P^T solve(P S h)
  launch_permute_in(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_h.p, n, h->d_xp.p);
  if (f32) run_solve<float>(h, 1, true); else run_solve<double>(h, 1, true);
  launch_permute_out(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_xp.p, nullptr, 0, h->d_w.p, n, 0);
  // FP64 residual and refinement
  launch_norm2(st, n, h->d_h.p, h->d_red.p, h->d_norm.p);
  double hn = 0.0;
  HIPCHK(h, hipMemcpyAsync(&hn, h->d_norm.p, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  if (hn == 0.0) hn = 1.0;
  int it = 0;
  double rel = 0.0;
  const int maxit = std::max(0, max_refine);
  while (true) {
    prof_launch(h, KC_RESID, 2.0 * h->nnzq, 0.0, [&] {
      launch_resid(st, n, h->d_qrp.p, h->d_qci.p, h->d_qpost.p, h->d_h.p, h->d_w.p, h->d_r.p);
      launch_norm2(st, n, h->d_r.p, h->d_red.p, h->d_norm.p);
    });
    double rn = 0.0;
    HIPCHK(h, hipMemcpyAsync(&rn, h->d_norm.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    rel = rn / hn;
    if (rel <= tol || it >= maxit || !std::isfinite(rel)) break;
    launch_permute_in(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_r.p, n, h->d_xp.p);
    if (f32) run_solve<float>(h, 1, true); else run_solve<double>(h, 1, true);
    launch_permute_out(st, n, 1, h->d_perm.p, h->d_scale.p, h->d_xp.p, nullptr, 0, h->d_w.p, n, 1);
    ++it;
  }
  // mu_post = mu + w
  launch_add(st, n, h->d_w.p, h->has_mu ? h->d_mu.p : nullptr, h->d_mu_post.p);
  HIPCHK(h, hipEventRecord(h->ev[3], st));
  h->ev_solve = true;
  HIPCHK(h, copy_d2d(mu_out, h->d_mu_post.p, n * sizeof(double), st));
  HIPCHK(h, hipStreamSynchronize(st));
  h->refine_iters = it;
  h->refine_resid = rel;
  if (iters_out) *iters_out = it;
  if (resid_out) *resid_out = rel;
  h->state |= ST_SOLVED;
  if (!(rel <= tol) && (f32 || maxit > 0)) {
    char msg[96];
    std::snprintf(msg, sizeof msg, "refinement stopped at relative residual %.3e after %d iterations", rel, it);
    return fail(h, GMRF_ERR_NOT_CONVERGED, msg);
  }
  return GMRF_OK;
}

gmrf_status gmrf_lml_gradient(gmrf_t post, gmrf_t prior, int k, const double* dq, const double* da,
                              const double* dqeps, int max_refine, double tol, double* out, double* mu_out) {
  if (!post || !prior || !out || k < 0 || (k > 0 && !dq)) return fail(post, GMRF_ERR_ARG, "bad argument");
  if (post == prior) return fail(post, GMRF_ERR_ARG, "prior and posterior must be two contexts");
  if (!(post->state & ST_FACTORED) || !(prior->state & ST_FACTORED))
    return fail(post, GMRF_ERR_STATE, "gmrf_lml_gradient needs both contexts factored");
  if (prior->n != post->n || prior->nnzq != post->nnzq || prior->qrp != post->qrp || prior->qci != post->qci)
    return fail(post, GMRF_ERR_PATTERN, "prior and posterior contexts hold different patterns of Q");
  if (post->nblocks != 1 || prior->nblocks != 1)
    return fail(post, GMRF_ERR_ARG, "gmrf_lml_gradient takes single-block contexts");
  if (prior->m != 0) return fail(post, GMRF_ERR_ARG, "the prior context must hold no observations");
  const int64_t n = post->n, nq = post->nnzq, m = post->m;
  // workspace: sig0, sig1, dqpost (nnz_q); mu, tmp, var (n); r, w, t1, t2, ones (m); scalars
  const int64_t ns = 8 + 8 * (int64_t)k;
  HIPCHK(post, post->d_lml.alloc((size_t)(3 * nq + 3 * n + 5 * std::max<int64_t>(m, 1) + ns)));
  double* sig0 = post->d_lml.p;
  double* sig1 = sig0 + nq;
  double* dqp = sig1 + nq;
  double* mu = dqp + nq;
  double* tmp = mu + n;
  double* var = tmp + n;
  double* r = var + n;
  double* w = r + std::max<int64_t>(m, 1);
  double* t1 = w + std::max<int64_t>(m, 1);
  double* t2 = t1 + std::max<int64_t>(m, 1);
  double* ones = t2 + std::max<int64_t>(m, 1);
  double* sc = ones + std::max<int64_t>(m, 1);
  double ld0 = 0.0, ld1 = 0.0;
  gmrf_status rc = gmrf_logdet(prior, &ld0);
  if (rc != GMRF_OK) return fail(post, rc, std::string("prior: ") + gmrf_last_error(prior));
  rc = gmrf_logdet(post, &ld1);
  if (rc != GMRF_OK) return rc;
  int iters = 0;
  double res = 0.0;
  const gmrf_status solve_rc = gmrf_solve(post, mu, max_refine, tol, &iters, &res);
  if (solve_rc != GMRF_OK && solve_rc != GMRF_ERR_NOT_CONVERGED) return solve_rc;
  if (k > 0) {
    rc = gmrf_selinv(prior, var, sig0);   // Sigma of the prior on Q's pattern
    if (rc != GMRF_OK) return fail(post, rc, std::string("prior: ") + gmrf_last_error(prior));
    rc = gmrf_selinv(post, var, sig1);
    if (rc != GMRF_OK) return rc;
  }
  hipStream_t st = post->stream;
  double* red = post->d_red.p;   // partial sums (allocated by gmrf_solve)
  // scalars: sc[0] mu^T Q mu, sc[1] r^T Q_eps r, sc[2] sum log q_eps; per parameter i at
  // sc[8 + 8i]: tr(Q^-1 dQ), tr(Q_post^-1 dQ_post), mu^T dQ mu, sum dq_eps / q_eps,
  // sum dq_eps r^2, (Q_eps r)^T dA mu
  launch_fill_f64(st, sc, ns, 0.0);
  launch_spmv(st, n, post->d_qrp.p, post->d_qci.p, post->d_qval.p, mu, tmp);
  launch_dot(st, n, mu, tmp, red, sc + 0);
  if (m > 0) {
    launch_fill_f64(st, ones, m, 1.0);
    // r = y - b - A mu, w = Q_eps r
    launch_obs_resid_plain(st, m, post->d_arp.p, post->d_aci.p, post->d_aval.p, post->d_y.p,
                           post->has_b ? post->d_b.p : nullptr, mu, r);
    launch_elementwise(st, m, 0, post->d_qeps.p, r, w);
    launch_dot(st, m, w, r, red, sc + 1);
    launch_elementwise(st, m, 2, post->d_qeps.p, nullptr, t2);
    launch_dot(st, m, t2, ones, red, sc + 2);
  }
  for (int i = 0; i < k; ++i) {
    const double* dqi = dq + (int64_t)i * nq;
    const double* dai = da ? da + (int64_t)i * post->nnza : nullptr;
    const double* dei = dqeps ? dqeps + (int64_t)i * m : nullptr;
    double* g = sc + 8 + 8 * i;
    launch_dot(st, nq, sig0, dqi, red, g + 0);
    launch_assemble_dqpost(st, nq, dqi, post->d_cptr.p, post->d_cpair.p, post->d_arow.p, post->d_aval.p,
                           m > 0 ? dai : nullptr, post->d_qeps.p, m > 0 ? dei : nullptr, dqp);
    launch_dot(st, nq, sig1, dqp, red, g + 1);
    launch_spmv(st, n, post->d_qrp.p, post->d_qci.p, dqi, mu, tmp);
    launch_dot(st, n, mu, tmp, red, g + 2);
    if (m > 0 && dei) {
      launch_elementwise(st, m, 1, dei, post->d_qeps.p, t1);
      launch_dot(st, m, t1, ones, red, g + 3);
      launch_elementwise(st, m, 0, dei, r, t1);
      launch_dot(st, m, t1, r, red, g + 4);
    }
    if (m > 0 && dai) {
      launch_spmv_obs(st, m, post->d_arp.p, post->d_aci.p, dai, mu, t1);
      launch_dot(st, m, w, t1, red, g + 5);
    }
  }
  HIPCHK(post, hipGetLastError());
  std::vector<double> hs((size_t)ns);
  HIPCHK(post, hipMemcpyAsync(hs.data(), sc, ns * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(post, hipStreamSynchronize(st));
  const double kLog2Pi = 1.8378770664093454836;
  out[0] = -0.5 * (double)m * kLog2Pi + 0.5 * ld0 + 0.5 * hs[2] - 0.5 * ld1 - 0.5 * hs[0] - 0.5 * hs[1];
  for (int i = 0; i < k; ++i) {
    const double* g = hs.data() + 8 + 8 * i;
    out[1 + i] = 0.5 * g[0] + 0.5 * g[3] - 0.5 * g[1] - 0.5 * g[2] - 0.5 * g[4] + g[5];
  }
  if (mu_out) {
    HIPCHK(post, copy_d2d(mu_out, mu, n * sizeof(double), st));
    HIPCHK(post, hipStreamSynchronize(st));
  }
  return solve_rc;
}

gmrf_status gmrf_pcg(gmrf_t h, int64_t k, const double* rhs, const double* x0, double* x_out, int precond, int maxit,
                     double tol, int* iters_out, double* resid_out) {
  if (!h || !x_out || k < 1 || maxit < 0 || !(tol >= 0.0) || (!rhs && k != 1)) return fail(h, GMRF_ERR_ARG, "bad argument");
  HIPCHK(h, sel_sync(h));
  gmrf_status rc = pcg_prepare(h, precond);
  if (rc != GMRF_OK) return rc;
  hipStream_t st = h->stream;
  const int64_t n = h->n;
  bool conv = true;
  for (int64_t c = 0; c < k; ++c) {
    double* x = x_out + c * n;
    const double* b = rhs ? rhs + c * n : h->d_h.p;
    if (x0) HIPCHK(h, copy_d2d(x, x0 + c * n, n * sizeof(double), st));
    int its = 0;
    double rel = 0.0;
    if (precond == 1 && h->prec == GMRF_FP32_REFINE) pcg_solve<float>(h, b, x, x0 != nullptr, precond, maxit, tol, &its, &rel);
    else pcg_solve<double>(h, b, x, x0 != nullptr, precond, maxit, tol, &its, &rel);
    if (!rhs && h->has_mu) launch_add(st, n, x, h->d_mu.p, x);   // posterior mean = mu + Q_post^-1 h
    if (iters_out) iters_out[c] = its;
    if (resid_out) resid_out[c] = rel;
    conv = conv && rel <= tol;
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(st));
  if (!conv) return fail(h, GMRF_ERR_NOT_CONVERGED, "conjugate gradients stopped above the tolerance");
  return GMRF_OK;
}

gmrf_status gmrf_sample_cg(gmrf_t h, int64_t k, int64_t r, const int64_t* r_rowptr, const int32_t* r_col,
                           const double* r_val, const double* w1, const double* w2, double* x_out, int precond,
                           int maxit, double tol, int* iters_out) {
  if (!h || k < 1 || r < 1 || !r_rowptr || !r_col || !r_val || !w1 || !x_out || (h->m > 0 && !w2))
    return fail(h, GMRF_ERR_ARG, "bad argument");
  if (!(h->state & ST_SOLVED)) return fail(h, GMRF_ERR_STATE, "gmrf_sample_cg needs a posterior mean (gmrf_solve)");
  HIPCHK(h, sel_sync(h));
  gmrf_status rc = pcg_prepare(h, precond);
  if (rc != GMRF_OK) return rc;
  hipStream_t st = h->stream;
  const int64_t n = h->n, m = h->m;
  HIPCHK(h, h->d_rvec.alloc((size_t)std::max<int64_t>(m, 1)));
  bool conv = true;
  for (int64_t c = 0; c < k; ++c) {
    double* x = x_out + c * n;
    // b = R w1 + A^T Q_eps^1/2 w2: covariance R R^T + A^T Q_eps A = Q_post
    double* b = h->d_w.p;
    launch_spmv(st, n, r_rowptr, r_col, r_val, w1 + c * r, b);
    if (m > 0) {
      launch_elementwise(st, m, 3, h->d_qeps.p, w2 + c * m, h->d_rvec.p);
      launch_at_times(st, n, h->d_atp.p, h->d_ati.p, h->d_arow.p, h->d_aval.p, h->d_rvec.p, h->d_r.p);
      launch_add(st, n, b, h->d_r.p, b);
    }
    int its = 0;
    double rel = 0.0;
    if (precond == 1 && h->prec == GMRF_FP32_REFINE) pcg_solve<float>(h, b, x, false, precond, maxit, tol, &its, &rel);
    else pcg_solve<double>(h, b, x, false, precond, maxit, tol, &its, &rel);
    launch_add(st, n, x, h->d_mu_post.p, x);
    if (iters_out) iters_out[c] = its;
    conv = conv && rel <= tol;
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(st));
  if (!conv) return fail(h, GMRF_ERR_NOT_CONVERGED, "conjugate gradients stopped above the tolerance");
  return GMRF_OK;
}

gmrf_status gmrf_rbmc_variances(gmrf_t h, int64_t k, const double* xs, double* var_out) {
  if (!h || k < 1 || !xs || !var_out) return fail(h, GMRF_ERR_ARG, "bad argument");
  if (!(h->state & ST_ASSEMBLED)) return fail(h, GMRF_ERR_STATE, "gmrf_rbmc_variances before gmrf_assemble");
  launch_rbmc(h->stream, h->n, h->d_qrp.p, h->d_qci.p, h->d_qpost.p, h->d_qdiag.p, k, xs, var_out);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return GMRF_OK;
}

gmrf_status gmrf_solve_rhs(gmrf_t h, const double* rhs, double* x_out) {
  if (!h || !rhs || !x_out) return fail(h, GMRF_ERR_ARG, "null argument");
  if (!(h->state & ST_FACTORED)) return fail(h, GMRF_ERR_STATE, "gmrf_solve_rhs before gmrf_factor");
  gmrf_status rc = check_status(h);
  if (rc != GMRF_OK) return rc;
  rc = alloc_solve(h, 1);
  if (rc != GMRF_OK) return rc;
  hipStream_t st = h->stream;
  launch_permute_in(st, h->n, 1, h->d_perm.p, h->d_scale.p, rhs, h->n, h->d_xp.p);
  if (h->prec == GMRF_FP32_REFINE) run_solve<float>(h, 1, true);
  else run_solve<double>(h, 1, true);
  launch_permute_out(st, h->n, 1, h->d_perm.p, h->d_scale.p, h->d_xp.p, nullptr, 0, x_out, h->n, 0);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(st));
  return GMRF_OK;
}

gmrf_status gmrf_gn_burgers(gmrf_t h, int64_t nx, int64_t nt, double dt, double nu, const double* mass,
                            const double* stiff3, int iters, int precision, int refine, double refine_tol,
                            double decrement_tol, int use_graph, double* u, double* rec_out) {
  if (!h || !mass || !stiff3 || !u || iters < 1 || refine < 0 || !(refine_tol >= 0.0) || !(decrement_tol >= 0.0))
    return fail(h, GMRF_ERR_ARG, "bad argument");
  HIPCHK(h, sel_sync(h));
  if (precision != GMRF_FP64 && precision != GMRF_FP32_REFINE) return fail(h, GMRF_ERR_ARG, "unknown precision");
  if (!(h->state & ST_ANALYZED)) return fail(h, GMRF_ERR_STATE, "gmrf_gn_burgers before gmrf_analyze");
  if (nx < 2 || nt < 2 || h->n != nx * nt || h->m != nx * nt || !(dt > 0.0))
    return fail(h, GMRF_ERR_ARG, "sizes do not match the assembled Burgers problem");
  // the rows of A must have the Burgers layout
  for (int64_t r = 0; r < h->m; ++r) {
    const int64_t e0 = h->arp[r], e1 = h->arp[r + 1];
    if (r < nx) {
      if (e1 - e0 != 1 || h->aci[e0] != r) return fail(h, GMRF_ERR_PATTERN, "A row " + std::to_string(r) + " is not an initial-condition row");
      continue;
    }
    const int64_t q = r - nx, k = q / nx + 1, i = q % nx;
    int64_t want[4], c = 0;
    want[c++] = (k - 1) * nx + i;
    if (i > 0) want[c++] = k * nx + i - 1;
    want[c++] = k * nx + i;
    if (i + 1 < nx) want[c++] = k * nx + i + 1;
    if (e1 - e0 != c) return fail(h, GMRF_ERR_PATTERN, "A row " + std::to_string(r) + " has the wrong length");
    for (int64_t t = 0; t < c; ++t)
      if (h->aci[e0 + t] != want[t]) return fail(h, GMRF_ERR_PATTERN, "A row " + std::to_string(r) + " has wrong columns");
  }
  GNArgs a{0, nx, nt, dt, nu, mass, stiff3, nullptr, nullptr, nullptr, 0, u, refine, refine_tol};
  return gn_run(h, a, iters, precision, use_graph, decrement_tol, rec_out);
}

gmrf_status gmrf_gn_pointwise(gmrf_t h, const double* lin_val, const int32_t* nl_col, const double* nl_coef,
                              int power, int iters, int precision, int refine, double refine_tol,
                              double decrement_tol, int use_graph, double* u, double* rec_out) {
  if (!h || !lin_val || !nl_col || !nl_coef || !u || iters < 1 || refine < 0 || !(refine_tol >= 0.0) ||
      !(decrement_tol >= 0.0) ||
      power < 2 || power > 8)
    return fail(h, GMRF_ERR_ARG, "bad argument");
  HIPCHK(h, sel_sync(h));
  if (precision != GMRF_FP64 && precision != GMRF_FP32_REFINE) return fail(h, GMRF_ERR_ARG, "unknown precision");
  if (!(h->state & ST_ANALYZED)) return fail(h, GMRF_ERR_STATE, "gmrf_gn_pointwise before gmrf_analyze");
  if (h->m < 1) return fail(h, GMRF_ERR_ARG, "gmrf_gn_pointwise needs observation rows");
  {
    // the nonlinear term's unknown must be a stored column of its row (its Jacobian entry)
    std::vector<int32_t> nc((size_t)h->m);
    HIPCHK(h, hipMemcpyAsync(nc.data(), nl_col, h->m * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int64_t r = 0; r < h->m; ++r) {
      if (nc[r] < 0) continue;
      if (nc[r] >= h->n || !std::binary_search(h->aci.begin() + h->arp[r], h->aci.begin() + h->arp[r + 1], nc[r]))
        return fail(h, GMRF_ERR_PATTERN, "nonlinear unknown of row " + std::to_string(r) + " is not in the row's pattern");
    }
  }
  GNArgs a{1, 0, 0, 0.0, 0.0, nullptr, nullptr, lin_val, nl_col, nl_coef, power, u, refine, refine_tol};
  return gn_run(h, a, iters, precision, use_graph, decrement_tol, rec_out);
}

gmrf_status gmrf_sample(gmrf_t h, int64_t k, const float* z, double* x_out) {
  if (!h || !z || !x_out) return fail(h, GMRF_ERR_ARG, "null argument");
  if (k < 1 || k > 16) return fail(h, GMRF_ERR_ARG, "k must be 1..16");
  if (!(h->state & ST_SOLVED)) return fail(h, GMRF_ERR_STATE, "gmrf_sample needs a posterior mean (gmrf_solve)");
  gmrf_status rc = check_status(h);
  if (rc != GMRF_OK) return rc;
  rc = alloc_solve(h, (int)k);
  if (rc != GMRF_OK) return rc;
  hipStream_t st = h->stream;
  launch_permute_in_f32(st, h->n, (int)k, z, h->d_xp.p);
  if (h->prec == GMRF_FP32_REFINE) run_solve<float>(h, (int)k, false);
  else run_solve<double>(h, (int)k, false);
  launch_permute_out(st, h->n, (int)k, h->d_perm.p, h->d_scale.p, h->d_xp.p, h->d_mu_post.p, 0, x_out, h->n, 0);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(st));
  return GMRF_OK;
}

gmrf_status gmrf_selinv_submit(gmrf_t h, double* var_out, double* sigma_q_out) {
  if (!h || !var_out) return fail(h, GMRF_ERR_ARG, "null argument");
  if (!(h->state & ST_FACTORED)) return fail(h, GMRF_ERR_STATE, "gmrf_selinv before gmrf_factor");
  HIPCHK(h, sel_sync(h));
  gmrf_status rc = check_status(h);
  if (rc != GMRF_OK) return rc;
  if (!h->sel_stream) {
    HIPCHK(h, hipStreamCreateWithFlags(&h->sel_stream, hipStreamNonBlocking));
    HIPCHK(h, hipEventCreateWithFlags(&h->ev_sel_start, hipEventDisableTiming));
    HIPCHK(h, hipEventCreateWithFlags(&h->ev_sel_done, hipEventDisableTiming));
  }
  // the inversion reads the factor and reuses the front buffers: order it after
  // everything already queued on the context's stream
  HIPCHK(h, hipEventRecord(h->ev_sel_start, h->stream));
  HIPCHK(h, hipStreamWaitEvent(h->sel_stream, h->ev_sel_start, 0));
  hipStream_t user = h->stream;
  h->stream = h->sel_stream;
  struct Restore { gmrf_t h; hipStream_t s; ~Restore() { h->stream = s; } } restore{h, user};
  HIPCHK(h, hipEventRecord(h->ev[4], h->stream));
  rc = h->prec == GMRF_FP32_REFINE ? run_selinv<float>(h, var_out, sigma_q_out)
                                   : run_selinv<double>(h, var_out, sigma_q_out);
  if (rc != GMRF_OK) return rc;
  HIPCHK(h, hipEventRecord(h->ev[5], h->stream));
  HIPCHK(h, hipEventRecord(h->ev_sel_done, h->stream));
  h->ev_sel = true;
  h->sel_inflight = true;
  return GMRF_OK;
}

gmrf_status gmrf_selinv_wait(gmrf_t h) {
  if (!h) return GMRF_ERR_ARG;
  HIPCHK(h, sel_sync(h));
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

gmrf_status gmrf_selinv(gmrf_t h, double* var_out, double* sigma_q_out) {
  gmrf_status rc = gmrf_selinv_submit(h, var_out, sigma_q_out);
  if (rc != GMRF_OK) return rc;
  return gmrf_selinv_wait(h);
}

gmrf_status gmrf_dot(gmrf_t h, int64_t len, const double* a, const double* b, double* out) {
  if (!h || !a || !b || !out || len < 0) return fail(h, GMRF_ERR_ARG, "bad argument");
  HIPCHK(h, h->d_red.alloc(1024));
  HIPCHK(h, h->d_norm.alloc(4));
  launch_dot(h->stream, len, a, b, h->d_red.p, h->d_norm.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(out, h->d_norm.p, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return GMRF_OK;
}

gmrf_status gmrf_matern_values(gmrf_t h, int64_t nnz, const double* m_on_q, const double* s_on_q,
                               const double* sms_on_q, double kappa, double tau, double* q_out, double* dq_out) {
  if (!h || nnz < 0 || !m_on_q || !s_on_q || !sms_on_q || !q_out) return fail(h, GMRF_ERR_ARG, "bad argument");
  if (!(kappa > 0.0) || !(tau > 0.0)) return fail(h, GMRF_ERR_ARG, "kappa and tau must be positive");
  launch_matern_values(h->stream, nnz, m_on_q, s_on_q, sms_on_q, kappa, tau, q_out, dq_out);
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

gmrf_status gmrf_spmv(gmrf_t h, const double* v_val, const double* x, double* y) {
  if (!h || !v_val || !x || !y) return fail(h, GMRF_ERR_ARG, "null argument");
  if (!(h->state & ST_ASSEMBLED)) return fail(h, GMRF_ERR_STATE, "gmrf_spmv before gmrf_assemble");
  launch_spmv(h->stream, h->n, h->d_qrp.p, h->d_qci.p, v_val, x, y);
  HIPCHK(h, hipGetLastError());
  return GMRF_OK;
}

gmrf_status gmrf_misfit(gmrf_t h, const double* x, double* out) {
  if (!h || !x || !out) return fail(h, GMRF_ERR_ARG, "null argument");
  if (!(h->state & ST_ASSEMBLED)) return fail(h, GMRF_ERR_STATE, "gmrf_misfit before gmrf_assemble");
  *out = 0.0;
  if (h->m == 0) return GMRF_OK;
  HIPCHK(h, h->d_red.alloc(1024));
  HIPCHK(h, h->d_norm.alloc(4));
  launch_weighted_resid(h->stream, h->m, h->d_arp.p, h->d_aci.p, h->d_aval.p, h->d_qeps.p, h->d_y.p,
                        h->has_b ? h->d_b.p : nullptr, x, h->d_rvec.p);
  launch_dot(h->stream, h->m, h->d_rvec.p, h->d_rvec.p, h->d_red.p, h->d_norm.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(out, h->d_norm.p, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return GMRF_OK;
}

static void fill_sym_stats(const Symbolic& Y, gmrf_stats_t* o) {
  o->n = Y.n;
  o->nnz_l = Y.nnzL;
  o->stored_l = Y.stored_L;
  o->n_super = Y.ns;
  o->tree_depth = Y.max_depth + 1;
  int64_t mf = 0;
  for (int32_t s = 0; s < Y.ns; ++s) mf = std::max<int64_t>(mf, Y.nf(s));
  o->max_front = mf;
  o->flops_factor = Y.flops_factor;
  o->flops_selinv = Y.flops_selinv;
  o->flops_solve = Y.flops_solve;
}

gmrf_status gmrf_stats(gmrf_t h, gmrf_stats_t* out) {
  if (!h || !out) return fail(h, GMRF_ERR_ARG, "null argument");
  std::memset(out, 0, sizeof(*out));
  out->failed_index = -1;
  gmrf_status rc = GMRF_OK;
  if (h->state & ST_FACTORED) rc = check_status(h);
  if (h->state & ST_ANALYZED) fill_sym_stats(h->sym, out);
  out->n = h->n;
  out->nnz_q = h->nnzq;
  out->m = h->m;
  out->nnz_a = h->nnza;
  const double w = h->prec == GMRF_FP32_REFINE ? 4.0 : 8.0;
  out->bytes_front_ws = (double)(h->sym.Wsize[0] + h->sym.Wsize[1]) * w;
  out->bytes_factor = (double)h->sym.Lsize * w;
  out->failed_index = h->failed_index;
  out->precision = h->prec;
  out->refine_iters = h->refine_iters;
  out->refine_resid = h->refine_resid;
  return rc;
}

gmrf_status gmrf_pivot_order(gmrf_t h, int32_t* perm_out) {
  if (!h || !perm_out) return fail(h, GMRF_ERR_ARG, "null argument");
  if (!(h->state & ST_ANALYZED)) return fail(h, GMRF_ERR_STATE, "gmrf_pivot_order before gmrf_analyze");
  std::memcpy(perm_out, h->sym.perm.data(), sizeof(int32_t) * h->n);
  return GMRF_OK;
}

gmrf_status gmrf_profile(gmrf_t h, int enable) {
  if (!h) return GMRF_ERR_ARG;
  prof_fold(h);
  for (int c = 0; c < KC_COUNT; ++c) { h->cls_ms[c] = 0; h->cls_flops[c] = 0; h->cls_bytes[c] = 0; h->cls_n[c] = 0; }
  h->recs.clear();
  h->prof = enable != 0;
  h->prof_mask = enable == 1 ? 0xffffffffu : (uint32_t)enable;
  return GMRF_OK;
}

gmrf_status gmrf_kernel_stats(gmrf_t h, gmrf_kernel_stat_t* out, int capacity, int* count) {
  if (!h) return GMRF_ERR_ARG;
  prof_fold(h);
  if (count) *count = KC_COUNT;
  if (!out) return GMRF_OK;
  for (int c = 0; c < KC_COUNT && c < capacity; ++c) {
    std::memset(out[c].name, 0, sizeof(out[c].name));
    std::strncpy(out[c].name, kClassNames[c], sizeof(out[c].name) - 1);
    out[c].launches = h->cls_n[c];
    out[c].ms = h->cls_ms[c];
    out[c].flops = h->cls_flops[c];
    out[c].bytes = h->cls_bytes[c];
  }
  return GMRF_OK;
}

gmrf_status gmrf_launch_records(gmrf_t h, gmrf_launch_rec_t* out, int64_t capacity, int64_t* count) {
  if (!h || capacity < 0) return fail(h, GMRF_ERR_ARG, "bad argument");
  prof_fold(h);
  if (count) *count = (int64_t)h->recs.size();
  if (out) {
    const size_t c = std::min((size_t)capacity, h->recs.size());
    if (c) std::memcpy(out, h->recs.data(), c * sizeof(gmrf_launch_rec_t));
  }
  return GMRF_OK;
}

gmrf_status gmrf_phase_ms(gmrf_t h, double* out3) {
  if (!h || !out3) return fail(h, GMRF_ERR_ARG, "null argument");
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, sel_sync(h));
  out3[0] = h->ev_factor ? elapsed(h->ev[0], h->ev[1]) : 0.0;
  out3[1] = h->ev_solve ? elapsed(h->ev[2], h->ev[3]) : 0.0;
  out3[2] = h->ev_sel ? elapsed(h->ev[4], h->ev[5]) : 0.0;
  return GMRF_OK;
}

gmrf_status gmrf_symbolic_host(int64_t n, const int64_t* rowptr, const int32_t* col, const double* coords, int dim,
                               const gmrf_options* opts, const int32_t* perm_in, int32_t* perm_out,
                               int64_t* colcount_out, gmrf_stats_t* stats_out) {
  if (n <= 0 || !rowptr || !col) return GMRF_ERR_ARG;
  std::vector<int64_t> rp(rowptr, rowptr + n + 1);
  std::vector<int32_t> ci(col, col + rp[n]);
  if (!check_csr(n, n, rp, ci, "Q").empty()) return GMRF_ERR_ARG;
  AnalyzeOptions opt;
  fill_opts(opts, opt);
  opt.nb = kNB;
  Symbolic Y;
  std::string e = analyze(n, rp.data(), ci.data(), coords, coords ? dim : 0, opt, Y, perm_in);
  if (!e.empty()) return GMRF_ERR_ARG;
  if (perm_out) std::memcpy(perm_out, Y.perm.data(), sizeof(int32_t) * n);
  if (colcount_out) std::memcpy(colcount_out, Y.colcount.data(), sizeof(int64_t) * n);
  if (stats_out) {
    std::memset(stats_out, 0, sizeof(*stats_out));
    fill_sym_stats(Y, stats_out);
    stats_out->nnz_q = rp[n];
    stats_out->failed_index = -1;
    stats_out->bytes_front_ws = 8.0 * (double)(Y.Wsize[0] + Y.Wsize[1]);
    stats_out->bytes_factor = 8.0 * (double)Y.Lsize;
  }
  return GMRF_OK;
}

}  // extern "C"
