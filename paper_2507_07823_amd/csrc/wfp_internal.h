// Internal plan state shared by the single-problem march, the gradient pass
// and the batched form.  Not part of the C ABI.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/wfp.h"
#include "wfp_host.h"
#include "wfp_kernels.h"

namespace wfpi {

using namespace wfp;


extern thread_local std::string g_last_error;

// mean neighbours per spring from which local_mode 0 (plans and batch
// instances) stores the weights once per unordered pair even where the
// per-pair weights fit (measured on one MI355X with the library's schedule:
// 22 % slower at 69 neighbours, 3-4 % faster at 101, 17 % at 138, 18 % at 207,
// 35 % at 1373)
constexpr double kPairOnceNeighbours = 96.0;

struct Error {
  wfp_status code;
  std::string msg;
};

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw Error{e_ == hipErrorOutOfMemory ? WFP_ENOMEM : WFP_EHIP,                    \
                  std::string(#expr) + ": " + hipGetErrorString(e_)};                   \
  } while (0)

inline void fail(wfp_status c, const std::string& m) { throw Error{c, m}; }

template <class T>
T* dalloc(size_t n, int64_t& counter) {
  T* p = nullptr;
  if (n == 0) n = 1;
  HIPCHK(hipMalloc(&p, n * sizeof(T)));
  counter += (int64_t)(n * sizeof(T));
  return p;
}

template <class T>
void upload(T* d, const std::vector<T>& h, hipStream_t s) {
  if (!h.empty()) HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Same mode position as the device (see mode_pos in the kernels).
inline int64_t mode_pos_host(int64_t q, int n1, int n2) {
  const int k2 = (int)(q % n2), k1 = (int)(q / n2);
  const int b = (k2 == 0) ? 0 : std::min(k2, n2 - k2);
  const int c = (k2 == b) ? 0 : 1;
  return (int64_t)b * 2 * n1 + c * n1 + k1;
}

// Inverse of a small dense matrix (row-major n x n) by Gauss-Jordan elimination
// with partial pivoting in long double.
inline void invert_dense(int n, const double* a, double* out) {
  std::vector<long double> m((size_t)n * 2 * n, 0.0L);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) m[(size_t)i * 2 * n + j] = a[(size_t)i * n + j];
    m[(size_t)i * 2 * n + n + i] = 1.0L;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs((double)m[(size_t)r * 2 * n + c]) > std::fabs((double)m[(size_t)piv * 2 * n + c])) piv = r;
    if (m[(size_t)piv * 2 * n + c] == 0.0L) fail(WFP_EDOMAIN, "singular per-step system");
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(m[(size_t)piv * 2 * n + j], m[(size_t)c * 2 * n + j]);
    const long double d = m[(size_t)c * 2 * n + c];
    for (int j = 0; j < 2 * n; ++j) m[(size_t)c * 2 * n + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const long double f = m[(size_t)r * 2 * n + c];
      if (f == 0.0L) continue;
      for (int j = 0; j < 2 * n; ++j) m[(size_t)r * 2 * n + j] -= f * m[(size_t)c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[(size_t)i * n + j] = (double)m[(size_t)i * 2 * n + n + j];
}

inline FftPlan make_fft_plan(int64_t n) {
  FftPlan fp{};
  fp.n = (int)n;
  std::vector<int> r = radix_sequence(n);
  if ((int)r.size() > kMaxFftStages) fail(WFP_EDOMAIN, "FFT length has too many stages");
  fp.nst = (int)r.size();
  for (size_t i = 0; i < r.size(); ++i) fp.radix[i] = r[i];
  for (int R : r)
    if (n / R > (int64_t)kFftMaxB * kFftThreads) fail(WFP_EDOMAIN, "FFT length too large for one workgroup");
  return fp;
}


wfp_status guard(const std::function<void()>& f);

}  // namespace wfpi

using namespace wfpi;

struct wfp_plan;
// Drops the plan's hold on its split's masked streams (destroyed with the
// last hold).  Never throws.
void release_overlap_streams(wfp_plan* P) noexcept;

struct wfp_plan {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t dev_bytes = 0;
  // sizes and parameters
  int64_t M = 0, R = 0, K = 0, level = 0, n_pairs = 0, n_pairs_recv = 0;
  int boundary = 0, W = 0, p = 0, NQ = 0, NH = 0, ngl = 0, ngpq = 0, rbc_period = 0, width = 0, iters = 0;
  int nf = 0, nfh = 0, ncheb = 0, T = 256, ntile = 0, ext_max = 0, npk = 0;
  double dt = 0, delta = 0, b = 0, hf = 0, alpha_es = 0, beta_es = 0, h_rbc = 0, delta_s = 0, contraction = 0;
  FftPlan fft_nf{}, fft_rbc{}, fft_n1{}, fft_n2{};
  // threads of the row passes (256, or 1024 for long rows)
  int hist_threads = 256;
  double* gsp = nullptr;    // spread grid of the 1024-thread row passes (nf)
  // FIR tap groups of the column pass and its LDS bytes
  int fir_groups = 8;
  size_t lds_b = 0;
  // boundary projection over workgroups for long grids: K = rbc_a rbc_b
  bool rbc_split = false;
  int rbc_a = 0, rbc_b = 0;
  FftPlan fft_rbc_a{}, fft_rbc_b{};
  double2 *rbc_z = nullptr, *rbc_t = nullptr;
  int n1 = 0, n2 = 0;           // four-step split of the half-length transform
  int64_t npos = 0;             // length of the per-mode arrays (mode-position order)
  double2 *T1 = nullptr, *V = nullptr;
  size_t lds_rbc = 0, lds_jac = 0, lds_qw = 0;
  std::vector<int> perm_h;
  // device buffers
  double *xs = nullptr, *beta = nullptr, *xr = nullptr, *packets = nullptr;
  int* perm = nullptr;
  double* hist = nullptr;
  double2 *ring = nullptr, *alpha = nullptr, *dalpha = nullptr;
  double *pk = nullptr, *qk = nullptr, *rot = nullptr, *dk1 = nullptr, *dk2 = nullptr;
  double2* tw = nullptr;
  double2* tw1 = nullptr;   // tw[n2 k1], k1 < n1 (the column pass's twiddle factor)
  double2* tw_rbc = nullptr;
  double2* ybuf = nullptr;
  double* grid2 = nullptr;
  double *rbc_u = nullptr, *rbc_v = nullptr;
  int *cstart = nullptr, *ccount = nullptr;
  int *nb_start = nullptr, *nb_count = nullptr;
  int64_t* qoff = nullptr;
  double* Q = nullptr;          // dense weights of the scatterer rows (plan set-up only)
  double* Qc = nullptr;         // packed weights of lags >= 1
  unsigned* ac = nullptr;       // per (row, lag) source range a | c << 16
  uint2* acx = nullptr;         // per (row, lag): (a | c << 16, packed offset within the row)
  int nqd = 0;                  // quads of lags per row (local-sum tasks per row)
  int64_t* rowbase = nullptr;   // packed offset of each row
  double* ginc = nullptr;       // -g_j(t_L), per row (set by the gradient pass's drive)
  // driving data of g_chunk consecutive levels from g_lvl0 (row L - g_lvl0)
  double* gbuf = nullptr;
  int g_chunk = 0;
  // set only during wfp_run_noalloc: the driving-data block and the finite
  // flag in the library's static per-device scratch array instead
  double* g_ext = nullptr;
  int g_ext_chunk = 0;
  int* flag_ext = nullptr;
  int64_t g_lvl0 = -1;
  double* loc = nullptr;        // local sum of lags >= 1, per row
  // solve tiles
  int *tile_r0 = nullptr, *tile_el = nullptr, *tile_g0 = nullptr, *tile_left = nullptr, *tile_n = nullptr;
  int *srow_g = nullptr, *srow_ptr = nullptr, *scol = nullptr;
  double *srow_dinv = nullptr, *sval = nullptr;
  int solve_threads = 64;
  // local weights evaluated on the fly (when the stored ones would not fit)
  bool otf = false;
  // local_mode 3: the on-the-fly layout (upper ranges, partials, lag-0
  // nearby weights) with the local sum's weights stored once per unordered
  // pair: per row and lag a run over the first sources of its upper range
  bool sym_stored = false;
  int64_t* sym_rb = nullptr;      // row j's first weight in sym_q
  uint2* sym_acx = nullptr;       // (count, offset within the row) per (row, lag)
  double* sym_q = nullptr;
  int64_t* sym_upb = nullptr;     // row j's first pair in sym_colpart
  double* sym_colpart = nullptr;  // per upper pair: the column term (row l's share)
  int2* sym_cov = nullptr;        // per row: first covering row below it, first wrapped one
  int sym_kmax = 0;               // longest lag-1 run of a row, less one
  double *otf_z = nullptr, *otf_w = nullptr, *phitab = nullptr, *half_beta = nullptr;
  double* halfs = nullptr;       // 1/2 per row (the local part without beta)
  // symmetric on-the-fly local sum: per row the unwrapped end of its upper
  // source range, per block of kOtfRows rows the end of their union and the
  // offset of its column sums in otf_part; the rows' own sums in otf_rowacc
  int* otf_up_end = nullptr;
  int* otf_blk_end = nullptr;
  int64_t* otf_part_off = nullptr;
  double* otf_part = nullptr;
  double* otf_rowacc = nullptr;
  // gradient pass with weights stored once per pair: the signed derivative
  // weights of each row's upper range (lags 0 .. NQ - 1, packed like sym_q),
  // the two sums' row and column terms, and a row scale of ones
  int sym_spl = 1;               // sources per lane of the pair-once kernels (1 or 2)
  int64_t otf_tot_part = 0;      // length of otf_part
  // gradient pass with the weights on the fly: the two derivative sums' row
  // and column terms and those of the next adjoint level's local sum (in the
  // layout of otf_rowacc / otf_part), and that sum per row
  double *otfd_row1 = nullptr, *otfd_row2 = nullptr, *otfd_part1 = nullptr, *otfd_part2 = nullptr;
  double *otfd_row3 = nullptr, *otfd_part3 = nullptr, *otfd_next = nullptr;
  int64_t* symd_rb = nullptr;
  uint2* symd_acx = nullptr;
  double *symd_q = nullptr, *symd_row1 = nullptr, *symd_row2 = nullptr, *symd_col1 = nullptr,
         *symd_col2 = nullptr, *symd_one = nullptr;
  double *otf_na = nullptr, *otf_nw = nullptr;
  int otf_nblk = 0;
  // stored weights: the lags >= 2 part of the local sum of level L, in
  // locb[L & 1] (its lag-1 part is added after sigma^{L-1} is solved)
  double* locb = nullptr;
  // rows of 16 lanes per lag take lsplit wavefronts; parts 1 .. lsplit - 1 of
  // level L's lags >= 2 sum go to locb2 + ((L & 1)(lsplit - 1) + q - 1) M
  double* locb2 = nullptr;
  int lsplit = 1;
  // lanes per lag in the local sum (16, or 8 / 4 when the lag blocks are short)
  int lgrp = 16;
  // concurrent history chain: masked streams for the chain (sb) and the rest
  // (sa), and sd on the same compute units as sa for the lags >= 2 part of the
  // next level's local sum
  int overlap_cus = 0;
  int overlap_held = 0;          // split whose shared masked streams this plan holds (0: none)
  hipStream_t sa = nullptr, sb = nullptr, sd = nullptr;
  hipEvent_t ev_solved = nullptr, ev_chain = nullptr, ev_join = nullptr;
  hipEvent_t ev_big[2] = {nullptr, nullptr};
  // global-sweep solve (when tiles do not fit in LDS)
  bool solve_global = false, g_wave = false;
  int *g_ptr = nullptr, *g_col = nullptr;
  double *g_val = nullptr, *g_dinv = nullptr, *g_rhs = nullptr, *g_xa = nullptr, *g_xb = nullptr;
  // direct solve of small runs
  int n_direct_tiles = 0;
  int *dt_g0 = nullptr, *dt_n = nullptr, *dt_p0 = nullptr, *pt_cs = nullptr, *pt_cn = nullptr;
  int64_t* pt_inv = nullptr;
  double* inv = nullptr;
  // precomputed spreading / interpolation weights
  int64_t* swoff = nullptr;
  double* sw = nullptr;
  int *i0s = nullptr, *ri0s = nullptr;
  double *iw = nullptr, *riw = nullptr;
  int *rnb_start = nullptr, *rnb_count = nullptr;
  int64_t* rqoff = nullptr;
  double* Qr = nullptr;
  double *cheb_phi = nullptr, *cheb_g = nullptr;
  int64_t n_weights_nonzero = 0, n_weights_stored = 0, n_weights_lag1 = 0;
  // host copies kept for the gradient pass set-up
  std::vector<double> xs_h, xr_h;
  std::vector<int> nbc_h, rnbs_h, rnbc_h;
  std::vector<int64_t> rqoff_h;
  int64_t dense_total = 0;
  double *glz_d = nullptr, *glw_d = nullptr, *lagw_d = nullptr;
  // checkpoints of the current run (state at levels c * ckpt_every, c >= 1);
  // ckpt_every < 0 records every level instead, in blocks of -ckpt_every levels
  int ckpt_every = 0;
  bool ck_from0 = true;          // the levels run so far started from level 0
  std::vector<char*> ckpts;
  size_t ckpt_bytes = 0;
  // recorded levels, block b = levels b C .. b C + C - 1 (C = -ckpt_every):
  // rec_sig[b] rows NQ - 1 + i = sigma^{bC+i} after the NQ - 1 levels before
  // the block (sorted order), rec_D[b] row i = the forward derivative term of
  // level bC + i (f' + d/dx u_H at the springs)
  std::vector<double*> rec_sig, rec_D;
  // gradient pass: replay and adjoint states, per-segment buffers
  bool grad_ready = false, gradx_ready = false;
  double *rhist = nullptr, *ahist = nullptr;
  double2 *rring = nullptr, *ralpha = nullptr, *rdalpha = nullptr;
  double2 *aring = nullptr, *aalpha = nullptr, *adalpha = nullptr;
  double *segsig = nullptr, *segD = nullptr, *gb_acc = nullptr, *gx_acc = nullptr;
  double *xloc = nullptr, *xw = nullptr, *fprime = nullptr, *gridd = nullptr, *esort = nullptr;
  double* xloc2 = nullptr;       // forward derivative local sum of the level being swept back
  double2* yd = nullptr;
  int *adj_ptr = nullptr, *adj_rr = nullptr, *adj_ri = nullptr;
  int *rsort = nullptr, *rcs = nullptr, *rcc = nullptr;
  int64_t* rwo = nullptr;
  double* rsw = nullptr;
  double* DQa = nullptr;         // signed derivative weights, lags >= 0, packed by row
  int64_t* drowbase = nullptr;
  uint2* acxd = nullptr;
  double* dQr = nullptr;         // receivers' signed derivative weights, layout of Qr
  std::vector<void*> owned;
  // per-stage event timing
  bool profiling = false;
  // finite-value check at the end of wfp_run
  bool check_finite = false;
  int* finite_flag = nullptr;
  double prof_ms[WFP_N_STAGES] = {};
  int64_t prof_n[WFP_N_STAGES] = {};
  struct Pending {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;

  ~wfp_plan() {
    // work queued on the plan's stream may still read its buffers
    (void)hipStreamSynchronize(stream);
    if (sa) (void)hipStreamSynchronize(sa);
    if (sb) (void)hipStreamSynchronize(sb);
    if (sd) (void)hipStreamSynchronize(sd);
    // sa, sb and sd are shared by the plans on the device with the same split;
    // the last one to let go destroys them
    release_overlap_streams(this);
    for (hipEvent_t e : {ev_solved, ev_chain, ev_join, ev_big[0], ev_big[1]})
      if (e) (void)hipEventDestroy(e);
    for (auto& q : pending) {
      (void)hipEventDestroy(q.a);
      (void)hipEventDestroy(q.b);
    }
    for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
    for (void* ptr : owned) (void)hipFree(ptr);
  }
  void release(void* ptr) {
    for (auto& o : owned)
      if (o == ptr) {
        (void)hipFree(o);
        o = nullptr;
      }
  }
  template <class T>
  T* alloc(size_t n) {
    T* ptr = dalloc<T>(n, dev_bytes);
    owned.push_back(ptr);
    return ptr;
  }
};
