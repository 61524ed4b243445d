// Plan creation, the level loop and the exported C ABI (include/wfp.h).
#include "wfp_internal.h"

#include <map>
#include <mutex>

namespace wfpi {
thread_local std::string g_last_error;
}  // namespace wfpi

// Device memory of wfp_run_noalloc: the block of driving-data levels (and the
// finite-check flag in its first 256 bytes), one copy per GPU, held until the
// process ends.  Host code uses the per-device address from
// hipGetSymbolAddress, never the array's name.
constexpr size_t kScratchDoubles = (size_t)1 << 20;            // 8 MiB
constexpr size_t kScratchHead = 32;                             // doubles before the driving data
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_ptr;

// Address of the current device's scratch array (looked up once per device).
static double* device_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) throw Error{WFP_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
  g_scratch_ptr[device] = (double*)ptr;
  return (double*)ptr;
}

// Masked streams per (device, split), shared by the plans that use the split
// and destroyed when the last of them lets go (each masked stream holds a
// hardware queue until it is destroyed).
struct MaskedStreams {
  std::array<hipStream_t, 3> st{nullptr, nullptr, nullptr};
  int holds = 0;
};
static std::mutex g_masked_mu;
static std::map<std::pair<int, int>, MaskedStreams> g_masked;

void release_overlap_streams(wfp_plan* P) noexcept {
  if (P->overlap_held <= 0) return;
  std::lock_guard<std::mutex> lock(g_masked_mu);
  auto it = g_masked.find(std::make_pair(P->device, P->overlap_held));
  if (it != g_masked.end() && --it->second.holds == 0) {
    for (hipStream_t q : it->second.st)
      if (q) {
        (void)hipStreamSynchronize(q);
        (void)hipStreamDestroy(q);
      }
    g_masked.erase(it);
  }
  P->overlap_held = 0;
  P->sa = P->sb = P->sd = nullptr;
}


namespace {

// wavefronts per row of the stored-weight local sum (rows of 16 lanes per
// lag); 2 measured fastest of 1 to 4 at M = 1e4, 1e5 and 1e6
constexpr int kLocalSplit = 2;
// mean upper-range length (sources per row, each pair once) from which the
// pair-once kernels take two consecutive sources per lane
constexpr int kSymPairedRange = 96;

void zero_state(wfp_plan* P) {
  auto fill = [&](double* ptr, int64_t n) {
    hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, P->stream, ptr, n, 0.0);
  };
  fill(P->hist, (int64_t)P->NH * P->M);
  fill((double*)P->ring, 2 * (int64_t)P->W * P->npos);
  fill((double*)P->alpha, 2 * P->npos);
  fill((double*)P->dalpha, 2 * P->npos);
  fill((double*)P->ybuf, 2 * (P->K + 1));
  HIPCHK(hipGetLastError());
  P->level = 0;
  P->ck_from0 = true;
}

// Host-only checks of the problem and parameters (no HIP call), so invalid
// input is reported before any device work.
void validate(const wfp_problem* prob, const wfp_params* par) {
  if (!prob || !par) fail(WFP_EINVAL, "NULL problem or params");
  if (prob->M < 1) fail(WFP_EINVAL, "M must be >= 1");
  if (prob->M > (int64_t)1 << 30) fail(WFP_EINVAL, "M too large");
  if (!prob->x || !prob->beta) fail(WFP_EINVAL, "x and beta are required");
  if (prob->boundary != WFP_PERIODIC && prob->boundary != WFP_FREE_SPACE) fail(WFP_EINVAL, "bad boundary");
  if (prob->n_packets < 1 || prob->n_packets > 64 || !prob->packets) fail(WFP_EINVAL, "need 1..64 packets");
  if (prob->R < 0 || (prob->R > 0 && !prob->x_recv)) fail(WFP_EINVAL, "bad receivers");
  if (!(par->dt > 0) || !std::isfinite(par->dt)) fail(WFP_EINVAL, "dt must be positive");
  if (par->eps_window < 0 || !(par->eps_window < 1) || par->gamma < 0 || !(par->gamma < 1))
    fail(WFP_EINVAL, "eps_window and gamma must lie in [0, 1)");
  if (par->W < 0 || par->K < 0 || par->n_gl_local < 0 || par->n_gl_pq < 0 || par->rbc_period < 0 ||
      par->solve_iters < 0 || par->local_mode < 0 || par->local_mode > 3)
    fail(WFP_EINVAL, "negative size parameter");
  if (par->checkpoint_every < -(1 << 20)) fail(WFP_EINVAL, "recording blocks of at most 2^20 levels");
  if (par->checkpoint_every < 0 && prob->boundary != WFP_PERIODIC)
    fail(WFP_EDOMAIN, "recorded levels (checkpoint_every < 0) serve the gradient pass, periodic box only");
  if (par->checkpoint_every < 0 && prob->R < 1)
    fail(WFP_EINVAL, "recorded levels (checkpoint_every < 0) serve the gradient pass, which needs receivers");
  const int p = par->p > 0 ? par->p : 8;
  if (par->p < 0 || p % 2 || p < 2 || p > kMaxP) fail(WFP_EINVAL, "p must be even, 2..12");
  for (int64_t j = 0; j < prob->M; ++j) {
    if (!std::isfinite(prob->x[j]) || !std::isfinite(prob->beta[j])) fail(WFP_EINVAL, "non-finite x or beta");
    if (!(prob->beta[j] > 0)) fail(WFP_EINVAL, "beta must be positive");
    if (prob->x[j] < -kPi || prob->x[j] >= kPi) fail(WFP_EINVAL, "x must lie in [-pi, pi)");
  }
  for (int64_t r = 0; r < prob->R; ++r)
    if (!std::isfinite(prob->x_recv[r]) || prob->x_recv[r] < -kPi || prob->x_recv[r] >= kPi)
      fail(WFP_EINVAL, "receiver outside [-pi, pi)");
  for (int i = 0; i < prob->n_packets * 5; ++i)
    if (!std::isfinite(prob->packets[i])) fail(WFP_EINVAL, "non-finite packet");
  for (int i = 0; i < prob->n_packets; ++i)
    if (!(prob->packets[5 * i + 2] > 0)) fail(WFP_EINVAL, "packet width must be positive");
  const double eps = par->eps_window > 0 ? par->eps_window : 1e-12;
  const double gamma = par->gamma > 0 ? par->gamma : 0.5;
  const double b = std::log(1.0 / eps);
  const int W = par->W > 0 ? par->W : (int)std::lround(2.0 * b / (kPi * gamma));
  if (W * par->dt >= kPi) fail(WFP_EDOMAIN, "delta = W dt must be < pi");
  if (par->K > 0 && (double)par->K * par->dt > kPi * (1 + 1e-14)) fail(WFP_EDOMAIN, "K dt must not exceed pi");
  if (std::floor(kPi / par->dt) < 1 && par->K == 0) fail(WFP_EDOMAIN, "K < 1 (dt too large)");
  if (prob->boundary == WFP_FREE_SPACE) {
    int64_t K = par->K;
    if (K == 0) {
      K = (int64_t)std::floor(kPi / par->dt);
      while (K > 1 && !is_pow2_pow5(2 * K)) --K;
    }
    const double h = kPi / (double)K;
    const double margin = 3.0 * std::max(W * par->dt, W * h);
    for (int64_t j = 0; j < prob->M; ++j)
      if (prob->x[j] < -kPi + margin || prob->x[j] > kPi - margin)
        fail(WFP_EDOMAIN, "free space: scatterer outside Omega");
    for (int64_t r = 0; r < prob->R; ++r)
      if (prob->x_recv[r] < -kPi + margin || prob->x_recv[r] > kPi - margin)
        fail(WFP_EDOMAIN, "free space: receiver outside Omega");
  }
}

hipEvent_t take_event(wfp_plan* P) {
  if (!P->free_events.empty()) {
    hipEvent_t e = P->free_events.back();
    P->free_events.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

void flush_profile(wfp_plan* P) {
  if (P->pending.empty()) return;
  for (auto& q : P->pending) HIPCHK(hipEventSynchronize(q.b));   // events live on two streams
  for (auto& q : P->pending) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, q.a, q.b));
    P->prof_ms[q.stage] += ms;
    P->prof_n[q.stage] += 1;
    P->free_events.push_back(q.a);
    P->free_events.push_back(q.b);
  }
  P->pending.clear();
}

// Brackets one stage's kernels with events when profiling is on.
struct StageTimer {
  wfp_plan* P;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  StageTimer(wfp_plan* p, int stg, hipStream_t stream) : P(p), stage(stg), st(stream) {
    if (P->profiling) {
      a = take_event(P);
      HIPCHK(hipEventRecord(a, st));
    }
  }
  ~StageTimer() noexcept(false) {
    if (P->profiling) {
      hipEvent_t b = take_event(P);
      HIPCHK(hipEventRecord(b, st));
      P->pending.push_back({stage, a, b});
      if (P->pending.size() >= 1024) flush_profile(P);
    }
  }
};

constexpr int kQwThreads = 128;

// Local weights (deriv = 0) or their signed distance derivatives (deriv = 1)
// of `nrows` target rows against the sorted scatterers.
void launch_local_weights(wfp_plan* P, int nrows, const double* xt, const int* st, const int* cnt,
                          const int64_t* off, const double* scale, int deriv, const int64_t* pbs,
                          signed char* ml, double* Qd, int nq_out = -1) {
  if (nq_out < 0) nq_out = P->NQ;
  if (nrows == 0) return;
  const int periodic = P->boundary == WFP_PERIODIC ? 1 : 0;
#define WFP_QW(PP)                                                                                      \
  hipLaunchKernelGGL(k_local_weights<PP>, dim3(nrows), dim3(kQwThreads), P->lds_qw, P->stream, nrows, xt,  \
                     P->xs, (int)P->M, st, cnt, off, scale, periodic, P->dt, P->delta, P->W, P->NQ, P->ngl,  \
                     P->glz_d, P->glw_d, P->cheb_phi, P->cheb_g, P->ncheb, deriv, P->lagw_d, pbs, ml, nq_out, Qd)
  switch (P->p) {
    case 2: WFP_QW(2); break;
    case 4: WFP_QW(4); break;
    case 6: WFP_QW(6); break;
    case 8: WFP_QW(8); break;
    case 10: WFP_QW(10); break;
    default: WFP_QW(12); break;
  }
#undef WFP_QW
  HIPCHK(hipGetLastError());
}

// The concurrent schedule's streams for a split of `cus` compute units: the
// chain (sb) and the solve (sa) on the first cus, the local sum and driving
// data (sd) on the rest; cus <= 0 selects one stream.
void set_overlap(wfp_plan* P, int cus) {
  if (cus == P->overlap_held && cus > 0) {
    P->overlap_cus = cus;
    return;
  }
  // work of the previous split is finished before its streams may go
  if (P->sa) HIPCHK(hipStreamSynchronize(P->sa));
  if (P->sb) HIPCHK(hipStreamSynchronize(P->sb));
  if (P->sd) HIPCHK(hipStreamSynchronize(P->sd));
  release_overlap_streams(P);
  if (cus <= 0) {
    P->overlap_cus = -1;
    return;
  }
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, P->device));
  const int ncu = prop.multiProcessorCount;
  if (cus >= ncu) fail(WFP_EINVAL, "overlap_cus must be below the number of compute units");
  const int words = (ncu + 31) / 32;
  std::vector<uint32_t> ma(words, 0u), mb(words, 0u), md(words, 0u);
  for (int c = 0; c < ncu; ++c) {
    if (c < cus) {
      mb[c / 32] |= 1u << (c % 32);
      ma[c / 32] |= 1u << (c % 32);
    } else {
      md[c / 32] |= 1u << (c % 32);
    }
  }
  {
    std::lock_guard<std::mutex> lock(g_masked_mu);
    auto key = std::make_pair(P->device, cus);
    auto it = g_masked.find(key);
    if (it == g_masked.end()) {
      MaskedStreams ms;
      HIPCHK(hipExtStreamCreateWithCUMask(&ms.st[0], (uint32_t)words, ma.data()));
      HIPCHK(hipExtStreamCreateWithCUMask(&ms.st[1], (uint32_t)words, mb.data()));
      HIPCHK(hipExtStreamCreateWithCUMask(&ms.st[2], (uint32_t)words, md.data()));
      it = g_masked.emplace(key, ms).first;
    }
    ++it->second.holds;
    P->overlap_held = cus;
    P->sa = it->second.st[0];
    P->sb = it->second.st[1];
    P->sd = it->second.st[2];
  }
  if (!P->ev_solved) {
    HIPCHK(hipEventCreateWithFlags(&P->ev_solved, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ev_chain, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ev_big[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&P->ev_big[1], hipEventDisableTiming));
  }
  P->overlap_cus = cus;
}

void build(wfp_plan* P, const wfp_problem* prob, const wfp_params* par) {
  validate(prob, par);
  const int64_t M = prob->M;
  if (M < 1) fail(WFP_EINVAL, "M must be >= 1");
  if (M > (int64_t)1 << 30) fail(WFP_EINVAL, "M too large");
  if (!prob->x || !prob->beta) fail(WFP_EINVAL, "x and beta are required");
  if (prob->boundary != WFP_PERIODIC && prob->boundary != WFP_FREE_SPACE) fail(WFP_EINVAL, "bad boundary");
  if (prob->n_packets < 1 || prob->n_packets > 64 || !prob->packets) fail(WFP_EINVAL, "need 1..64 packets");
  if (prob->R < 0 || (prob->R > 0 && !prob->x_recv)) fail(WFP_EINVAL, "bad receivers");
  if (!(par->dt > 0) || !std::isfinite(par->dt)) fail(WFP_EINVAL, "dt must be positive");
  const bool periodic = prob->boundary == WFP_PERIODIC;
  P->M = M;
  P->R = prob->R;
  P->ckpt_every = par->checkpoint_every;
  P->check_finite = par->check_finite != 0;
  P->overlap_cus = par->overlap_cus;
  P->boundary = prob->boundary;
  P->dt = par->dt;
  const double eps = par->eps_window > 0 ? par->eps_window : 1e-12;
  const double gamma = par->gamma > 0 ? par->gamma : 0.5;
  P->b = std::log(1.0 / eps);
  P->W = par->W > 0 ? par->W : (int)std::lround(2.0 * P->b / (kPi * gamma));
  P->p = par->p > 0 ? par->p : 8;
  if (P->p % 2 || P->p < 2 || P->p > kMaxP) fail(WFP_EINVAL, "p must be even, 2..12");
  if (P->W + P->p / 2 > 64) fail(WFP_EDOMAIN, "W + p/2 must not exceed 64");
  P->delta = P->W * P->dt;
  if (P->delta >= kPi) fail(WFP_EDOMAIN, "delta = W dt must be < pi");
  if (par->K > 0) {
    P->K = par->K;
  } else {
    int64_t k = (int64_t)std::floor(kPi / P->dt);
    if (!periodic)
      while (k > 1 && !is_pow2_pow5(2 * k)) --k;
    P->K = k;
  }
  if (P->K < 1) fail(WFP_EDOMAIN, "K < 1 (dt too large)");
  if ((double)P->K * P->dt > kPi * (1 + 1e-14)) fail(WFP_EDOMAIN, "K dt must not exceed pi");
  P->NQ = P->W + P->p / 2;   // lags m = 0..W-1+p/2 carry weights
  P->NH = P->NQ;             // density levels kept: sigma^{L-1} .. sigma^{L-NQ}
  P->ngl = par->n_gl_local > 0 ? par->n_gl_local : P->W;
  P->ngpq = par->n_gl_pq > 0 ? par->n_gl_pq : 32;
  P->width = par->nufft_width > 0 ? par->nufft_width : 16;
  if (P->width > 64 || P->width < 4) fail(WFP_EINVAL, "nufft_width must be 4..64");
  P->h_rbc = kPi / (double)P->K;
  P->delta_s = P->W * P->h_rbc;
  P->rbc_period = par->rbc_period > 0 ? par->rbc_period
                                      : (int)std::ceil(P->W * P->h_rbc / P->dt - 1e-12);
  // fine grid: the smallest even 2^a 5^b >= 2 (2K+1) whose half length
  // n = n1 n2 splits with n1 = the largest 2^a 5^b divisor not above sqrt(n)
  // or 256 (the column pass holds 38 n1 complex values in LDS) and
  // n2 <= 8192 (one row in LDS)
  auto split = [](int64_t n, int64_t& n1) {
    n1 = 0;
    for (int64_t d = 1; d * d <= n && d <= 256; ++d)
      if (n % d == 0 && is_pow2_pow5(d)) n1 = d;
    return n1 > 0 && n / n1 <= 8192;
  };
  int64_t nf = 2 * (2 * P->K + 1), n1s = 0;
  while (!(is_pow2_pow5(nf) && nf % 2 == 0 && split(nf / 2, n1s))) {
    ++nf;
    if (nf > ((int64_t)1 << 30)) fail(WFP_EDOMAIN, "fine grid too long for the four-step transform");
  }
  P->nf = (int)nf;
  P->nfh = (int)(nf / 2);
  P->hf = kTwoPi / (double)nf;
  P->alpha_es = 0.5 * P->width * P->hf;
  P->beta_es = 2.30 * P->width;
  {
    const int64_t n = P->nfh;
    P->n1 = (int)n1s;
    P->n2 = (int)(n / n1s);
    P->fft_n1 = make_fft_plan(P->n1);
    P->fft_n2 = make_fft_plan(P->n2);
    // rows of 1024 points or more run on 1024 threads: the n1 <= 256 row
    // blocks are then about one per compute unit, and 256 threads (4
    // wavefronts) cannot hide the latency of their gathers and FFT stages
    P->hist_threads = P->n2 >= 1024 ? 1024 : 256;
    for (int i = 0; i < P->fft_n2.nst; ++i)
      if (P->n2 / P->fft_n2.radix[i] > kFftMaxB * 256) P->hist_threads = 1024;
    P->npos = (int64_t)(P->n2 / 2 + 1) * 2 * P->n1;
    // batched LDS stages run on 256 threads with at most kFftMaxB butterflies each
    for (int i = 0; i < P->fft_n1.nst; ++i)
      if (2 * P->n1 / P->fft_n1.radix[i] > kFftMaxB * 256) fail(WFP_EDOMAIN, "four-step factor n1 too long");
    for (int i = 0; i < P->fft_n2.nst; ++i)
      if (P->n2 / P->fft_n2.radix[i] > kFftMaxB * P->hist_threads)
        fail(WFP_EDOMAIN, "four-step factor n2 too long");
  }
  if (!periodic) {
    if (!is_pow2_pow5(2 * P->K)) fail(WFP_EDOMAIN, "free space needs 2K = 2^a 5^b");
    // one workgroup holds the K complex points while they fit in LDS and no
    // stage needs more than kFftMaxB butterflies per thread; longer grids
    // split K = a b over workgroups (a the largest divisor not above sqrt(K))
    bool one = (size_t)P->K * sizeof(double2) <= 160 * 1024;
    for (int R : radix_sequence(P->K))
      if (P->K / R > (int64_t)kFftMaxB * kFftThreads) one = false;
    if (one) {
      P->fft_rbc = make_fft_plan(P->K);
      P->lds_rbc = (size_t)P->K * sizeof(double2);
    } else {
      int64_t a = 1;
      for (int64_t d = 1; d * d <= P->K; ++d)
        if (P->K % d == 0) a = d;
      const int64_t b = P->K / a;
      auto fits = [](int64_t n) {
        if (n * (int64_t)sizeof(double2) > 160 * 1024) return false;
        for (int R : radix_sequence(n))
          if (n / R > (int64_t)kFftMaxB * 256) return false;
        return true;
      };
      if (!fits(a) || !fits(b)) fail(WFP_EDOMAIN, "boundary projection grid too long");
      P->rbc_split = true;
      P->rbc_a = (int)a;
      P->rbc_b = (int)b;
      P->fft_rbc_a = make_fft_plan(a);
      P->fft_rbc_b = make_fft_plan(b);
    }
  }

  hipStream_t s = P->stream;
  // ---- scatterers: validate, sort ----
  std::vector<double> xh(prob->x, prob->x + M), bh(prob->beta, prob->beta + M);
  const double margin = 3.0 * std::max(P->delta, P->delta_s);
  const double olo = -kPi + margin, ohi = kPi - margin;
  for (int64_t j = 0; j < M; ++j) {
    if (!std::isfinite(xh[j]) || !std::isfinite(bh[j])) fail(WFP_EINVAL, "non-finite x or beta");
    if (!(bh[j] > 0)) fail(WFP_EINVAL, "beta must be positive");
    if (xh[j] < -kPi || xh[j] >= kPi) fail(WFP_EINVAL, "x must lie in [-pi, pi)");
    if (!periodic && (xh[j] < olo || xh[j] > ohi)) fail(WFP_EDOMAIN, "free space: scatterer outside Omega");
  }
  std::vector<double> xrh(prob->x_recv ? prob->x_recv : nullptr, prob->x_recv ? prob->x_recv + P->R : nullptr);
  for (double v : xrh) {
    if (!std::isfinite(v) || v < -kPi || v >= kPi) fail(WFP_EINVAL, "receiver outside [-pi, pi)");
    if (!periodic && (v < olo || v > ohi)) fail(WFP_EDOMAIN, "free space: receiver outside Omega");
  }
  for (int i = 0; i < prob->n_packets * 5; ++i)
    if (!std::isfinite(prob->packets[i])) fail(WFP_EINVAL, "non-finite packet");
  for (int i = 0; i < prob->n_packets; ++i)
    if (!(prob->packets[5 * i + 2] > 0)) fail(WFP_EINVAL, "packet width must be positive");
  std::vector<int> perm(M);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int c) { return xh[a] < xh[c]; });
  std::vector<double> xs(M), bs(M);
  for (int64_t i = 0; i < M; ++i) {
    xs[i] = xh[perm[i]];
    bs[i] = bh[perm[i]];
  }
  P->perm_h = perm;
  P->xs_h = xs;

  // ---- window series, Gauss-Legendre rules ----
  WindowSeries ws = window_series(P->b, 128);
  P->ncheb = ws.n;
  {
    const double one = cheb_eval(ws.phi.data(), ws.n, 1.0);
    if (std::fabs(one - 1.0) > 1e-13) fail(WFP_EDOMAIN, "window series not normalised");
  }
  std::vector<double> glz, glw, gqz, gqw, gez, gew;
  gauss_legendre(P->ngl, glz, glw);
  gauss_legendre(P->ngpq, gqz, gqw);
  gauss_legendre(256, gez, gew);

  // ---- device allocations ----
  P->xs = P->alloc<double>(M);
  P->beta = P->alloc<double>(M);
  P->perm = P->alloc<int>(M);
  P->hist = P->alloc<double>((size_t)P->NH * M);
  P->ring = P->alloc<double2>((size_t)P->W * P->npos);
  P->alpha = P->alloc<double2>(P->npos);
  P->dalpha = P->alloc<double2>(P->npos);
  P->pk = P->alloc<double>((size_t)P->W * P->npos);
  P->qk = P->alloc<double>((size_t)P->W * P->npos);
  P->rot = P->alloc<double>(3 * P->npos);
  P->dk1 = P->alloc<double>(P->npos);
  P->dk2 = P->alloc<double>(P->npos);
  P->tw = P->alloc<double2>(nf);
  P->T1 = P->alloc<double2>(P->nfh);
  P->V = P->alloc<double2>(P->nfh);
  P->ybuf = P->alloc<double2>(P->K + 1);
  P->grid2 = P->alloc<double>(nf);
  if (P->hist_threads == 1024) P->gsp = P->alloc<double>(nf);
  P->cstart = P->alloc<int>(nf);
  P->ccount = P->alloc<int>(nf);
  P->cheb_phi = P->alloc<double>(ws.n);
  P->cheb_g = P->alloc<double>(ws.n);
  P->packets = P->alloc<double>(5 * prob->n_packets);
  P->npk = prob->n_packets;
  upload(P->xs, xs, s);
  upload(P->beta, bs, s);
  upload(P->perm, perm, s);
  upload(P->cheb_phi, ws.phi, s);
  upload(P->cheb_g, ws.g, s);
  upload(P->packets, std::vector<double>(prob->packets, prob->packets + 5 * prob->n_packets), s);

  // ---- twiddles e^{-2 pi i t / nf} ----
  {
    std::vector<double2> tw(nf);
    for (int64_t t = 0; t < nf; ++t) {
      const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)nf;
      tw[t] = make_double2((double)std::cos(a), (double)std::sin(a));
    }
    upload(P->tw, tw, s);
    std::vector<double2> tw1(P->n1);
    for (int k1 = 0; k1 < P->n1; ++k1) tw1[k1] = tw[(int64_t)P->n2 * k1];
    P->tw1 = P->alloc<double2>(P->n1);
    upload(P->tw1, tw1, s);
  }
  // ---- NUFFT deconvolution: Psi_hat(k) = alpha int_{-1}^{1} psi(z) cos(k alpha z) dz ----
  {
    std::vector<double> d1(P->npos, 0.0), d2(P->npos, 0.0), psi(256);
    for (int q = 0; q < 256; ++q) psi[q] = std::exp(P->beta_es * (std::sqrt(1.0 - gez[q] * gez[q]) - 1.0));
    for (int64_t k = 0; k <= P->K; ++k) {
      long double acc = 0;
      for (int q = 0; q < 256; ++q) acc += (long double)gew[q] * psi[q] * std::cos((double)k * P->alpha_es * gez[q]);
      const double ph = P->alpha_es * (double)acc;
      const double sg = (k & 1) ? -1.0 : 1.0;
      const int64_t pos = mode_pos_host(k, P->n1, P->n2);
      d1[pos] = sg * P->hf / (kTwoPi * ph);
      d2[pos] = sg * P->hf / ph;
    }
    upload(P->dk1, d1, s);
    upload(P->dk2, d2, s);
  }
  // ---- p_k, q_k tables and the propagator ----
  {
    std::vector<double> mu(P->ngpq), wmu(P->ngpq), dph((size_t)P->W * P->ngpq), ddph((size_t)P->W * P->ngpq);
    for (int q = 0; q < P->ngpq; ++q) {
      mu[q] = 0.5 * P->dt * (gqz[q] + 1.0);
      wmu[q] = 0.5 * P->dt * gqw[q];
    }
    for (int m = 0; m < P->W; ++m)
      for (int q = 0; q < P->ngpq; ++q) {
        const double tau = m * P->dt + mu[q];
        const double sv = 2.0 * tau / P->delta - 1.0;
        dph[m * P->ngpq + q] = (2.0 / P->delta) * cheb_eval(ws.g.data(), ws.n, sv);
        ddph[m * P->ngpq + q] = (4.0 / (P->delta * P->delta)) * cheb_eval(ws.dg.data(), ws.n, sv);
      }
    double* dmu = P->alloc<double>(P->ngpq);
    double* dwmu = P->alloc<double>(P->ngpq);
    double* ddph_d = P->alloc<double>(ddph.size());
    double* dph_d = P->alloc<double>(dph.size());
    upload(dmu, mu, s);
    upload(dwmu, wmu, s);
    upload(dph_d, dph, s);
    upload(ddph_d, ddph, s);
    hipLaunchKernelGGL(k_pq_tables, dim3(nblk(P->K + 1, 128)), dim3(128), 0, s, P->K, P->W, P->ngpq, P->dt,
                       dph_d, ddph_d, dmu, dwmu, P->n1, P->n2, P->npos, P->pk, P->qk, P->rot);
    HIPCHK(hipGetLastError());
  }
  // ---- spreading ranges: sources within the kernel support of each cell ----
  {
    std::vector<int> cs(nf), cc(nf);
    std::vector<int64_t> wo(nf);
    int64_t wt = 0;
    for (int64_t i = 0; i < nf; ++i) {
      const double xc = -kPi + (double)i * P->hf;
      source_range(xs, xc, P->alpha_es * (1.0 + 1e-12), true, true, cs[i], cc[i]);
      wo[i] = wt;
      wt += cc[i];
    }
    upload(P->cstart, cs, s);
    upload(P->ccount, cc, s);
    P->swoff = P->alloc<int64_t>(nf);
    P->sw = P->alloc<double>(wt);
    upload(P->swoff, wo, s);
    hipLaunchKernelGGL(k_spread_weights, dim3(nblk(nf, 256)), dim3(256), 0, s, (int)nf, P->hf, 1.0 / P->alpha_es,
                       P->beta_es, P->xs, (int)M, P->cstart, P->ccount, P->swoff, P->sw);
    HIPCHK(hipGetLastError());
    P->i0s = P->alloc<int>(M);
    P->iw = P->alloc<double>((size_t)M * P->width);
    hipLaunchKernelGGL(k_interp_weights, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, (int)nf, P->hf,
                       1.0 / P->alpha_es, P->beta_es, P->width, P->xs, P->i0s, P->iw);
    HIPCHK(hipGetLastError());
  }
  // ---- neighbour rows of the scatterers and receivers ----
  std::vector<int> nbs(M), nbc(M), ns(M), nc(M);
  std::vector<int64_t> qo(M), pb(M);
  int64_t tot = 0;
  for (int64_t j = 0; j < M; ++j) {
    source_range(xs, xs[j], P->delta, periodic, false, nbs[j], nbc[j]);
    source_range(xs, xs[j], P->dt, periodic, false, ns[j], nc[j]);
    qo[j] = tot;
    pb[j] = P->n_pairs;
    tot += (int64_t)nbc[j] * P->NQ;
    P->n_pairs += nbc[j];
  }
  // stored weights (dense per pair during set-up, then packed) or on the fly
  {
    int mode = par->local_mode;
    if (mode == 0) {
      // once per unordered pair (about half the set-up array and packed
      // weights) when that fits and either the springs have enough neighbours
      // (there the halved stream outweighs the prefix runs' idle lanes: it
      // measured faster from about 100 neighbours per spring on) or the
      // per-pair weights would not fit; else per ordered pair when they fit;
      // else on the fly
      size_t fr = 0, to = 0;
      HIPCHK(hipMemGetInfo(&fr, &to));
      const double need = 8.0 * (double)tot * 1.7;
      const bool fits1 = need < 0.6 * (double)fr, fits3 = 0.5 * need < 0.6 * (double)fr;
      const bool dense = (double)P->n_pairs >= kPairOnceNeighbours * (double)M;
      if (fits3 && (dense || !fits1)) mode = 3;
      else if (fits1) mode = 1;
      else mode = 2;
    }
    P->otf = mode == 2 || mode == 3;
    P->sym_stored = mode == 3;
  }
  // on the fly: only the lag-0 weights of nearby pairs are stored (for the solve)
  std::vector<int64_t> qoN(M);
  int64_t totN = 0;
  for (int64_t j = 0; j < M; ++j) {
    qoN[j] = totN;
    totN += nc[j];
  }
  auto lag0 = [&](int64_t g, int64_t l) -> int64_t {
    return P->otf ? qoN[g] + (l - ns[g] + M) % M : qo[g] + (l - nbs[g] + M) % M;
  };
  P->nb_start = P->alloc<int>(M);
  P->nb_count = P->alloc<int>(M);
  P->qoff = P->alloc<int64_t>(M);
  int64_t* pbase = P->alloc<int64_t>(M);
  signed char* mlo = P->otf ? nullptr : P->alloc<signed char>(P->n_pairs);
  P->Q = P->alloc<double>(P->otf ? totN : tot);
  upload(P->nb_start, nbs, s);
  upload(P->nb_count, nbc, s);
  upload(P->qoff, qo, s);
  upload(pbase, pb, s);
  std::vector<double> lagw(P->p);
  {
    for (int r = 0; r < P->p; ++r) {
      double f = 1.0;
      for (int q = 0; q < P->p; ++q)
        if (q != r) f *= (double)(r - q);
      lagw[r] = 1.0 / f;
    }
  }
  double* lagw_d = P->alloc<double>(P->p);
  double* glz_d = P->alloc<double>(P->ngl);
  double* glw_d = P->alloc<double>(P->ngl);
  upload(lagw_d, lagw, s);
  upload(glz_d, glz, s);
  upload(glw_d, glw, s);
  P->lagw_d = lagw_d;
  P->glz_d = glz_d;
  P->glw_d = glw_d;
  P->nbc_h = nbc;
  P->dense_total = tot;
  std::vector<double> half_beta(M);
  for (int64_t j = 0; j < M; ++j) half_beta[j] = 0.5 * bs[j];
  double* hb_d = P->alloc<double>(M);
  upload(hb_d, half_beta, s);
  P->lds_qw = (size_t)P->NQ * kQwThreads * sizeof(double);
  auto launch_qw = [&](int nrows, const double* xt, const int* st, const int* cnt, const int64_t* off,
                       const double* scale, const int64_t* pbs, signed char* ml, double* Qd) {
    launch_local_weights(P, nrows, xt, st, cnt, off, scale, 0, pbs, ml, Qd);
  };
  int* near_start = P->alloc<int>(M);
  int* near_count = P->alloc<int>(M);
  int64_t* near_off = P->alloc<int64_t>(M);
  upload(near_start, ns, s);
  upload(near_count, nc, s);
  upload(near_off, qoN, s);
  if (P->otf) {
    launch_local_weights(P, (int)M, P->xs, near_start, near_count, near_off, hb_d, 0, nullptr, nullptr, P->Q, 1);
    // on-the-fly tables: GL nodes in ascending z (decreasing lag), the window
    // phi as kPhiPieces polynomials of degree kPhiDeg in the local variable
    std::vector<int> ord(P->ngl);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int c) { return glz[a] < glz[c]; });
    std::vector<double> za(P->ngl), wa(P->ngl);
    for (int q = 0; q < P->ngl; ++q) {
      za[q] = glz[ord[q]];
      wa[q] = glw[ord[q]];
    }
    if (P->ngl > 64) fail(WFP_EDOMAIN, "on-the-fly local weights take at most 64 quadrature nodes");
    std::vector<double> tab = window_pieces(ws, kPhiPieces, kPhiDeg);
    {
      // the table reproduces the series to rounding
      double worst = 0.0;
      for (int i = 0; i <= 20000; ++i) {
        const double u = -1.0 + 2.0 * i / 20000.0;
        int pc = (int)((u + 1.0) * (0.5 * kPhiPieces));
        pc = pc < 0 ? 0 : (pc >= kPhiPieces ? kPhiPieces - 1 : pc);
        const double tt = (u + 1.0) * (0.5 * kPhiPieces) - pc;
        double v = tab[(size_t)pc * (kPhiDeg + 1) + kPhiDeg];
        for (int k = kPhiDeg - 1; k >= 0; --k) v = std::fma(v, tt, tab[(size_t)pc * (kPhiDeg + 1) + k]);
        worst = std::max(worst, std::fabs(v - cheb_eval(ws.phi.data(), ws.n, u)));
      }
      if (worst > 1e-15) fail(WFP_EDOMAIN, "window table for the on-the-fly weights is not accurate");
    }
    // upper source ranges of the symmetric local sum (each unordered pair once)
    {
      std::vector<int> up, be;
      std::vector<int64_t> po;
      int64_t tot_part = 0;
      if (!upper_ranges(nbs, nbc, kOtfRows, up, be, po, tot_part))
        fail(WFP_EINVAL, "upper source ranges of the on-the-fly local sum are inconsistent");
      const int nb = (int)be.size();
      P->otf_nblk = nb;
      P->otf_up_end = P->alloc<int>(M);
      P->otf_blk_end = P->alloc<int>(nb);
      P->otf_part_off = P->alloc<int64_t>(nb);
      P->otf_part = P->alloc<double>(tot_part);
      P->otf_tot_part = tot_part;
      P->otf_rowacc = P->alloc<double>(M);
      upload(P->otf_up_end, up, s);
      upload(P->otf_blk_end, be, s);
      upload(P->otf_part_off, po, s);
      if (P->sym_stored) {
        // weights of each unordered pair once: row j against its upper range
        // [j, up[j]) (dense, lag-major, unscaled), then per lag the run of
        // sources that carry it (from the row itself), packed
        std::vector<int> ust(M), ucnt(M);
        std::vector<int64_t> uoff(M), upb(M);
        std::vector<double> ones(M, 1.0);
        int64_t tot_up = 0, np_up = 0;
        for (int64_t j = 0; j < M; ++j) {
          ust[j] = (int)j;
          ucnt[j] = up[j] - (int)j;
          if (ucnt[j] >= 65536) fail(WFP_EDOMAIN, "more than 65535 upper neighbours of one scatterer");
          uoff[j] = tot_up;
          upb[j] = np_up;
          tot_up += (int64_t)ucnt[j] * P->NQ;
          np_up += ucnt[j];
        }
        int* ust_d = P->alloc<int>(M);
        int* ucnt_d = P->alloc<int>(M);
        int64_t* uoff_d = P->alloc<int64_t>(M);
        int64_t* upb_d = P->alloc<int64_t>(M);
        double* ones_d = P->alloc<double>(M);
        signed char* umlo = P->alloc<signed char>(np_up);
        double* dense = P->alloc<double>(tot_up);
        unsigned* uac = P->alloc<unsigned>((size_t)M * P->NQ);
        upload(ust_d, ust, s);
        upload(ucnt_d, ucnt, s);
        upload(uoff_d, uoff, s);
        upload(upb_d, upb, s);
        upload(ones_d, ones, s);
        launch_local_weights(P, (int)M, P->xs, ust_d, ucnt_d, uoff_d, ones_d, 0, upb_d, umlo, dense);
        hipLaunchKernelGGL(k_row_ranges, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ,
                           ucnt_d, upb_d, umlo, uac);
        HIPCHK(hipGetLastError());
        std::vector<unsigned> ach((size_t)M * P->NQ);
        HIPCHK(hipMemcpyAsync(ach.data(), uac, ach.size() * sizeof(unsigned), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int64_t> rb(M);
        std::vector<uint2> acxh((size_t)M * P->NQ);
        int64_t packed = 0;
        for (int64_t j = 0; j < M; ++j) {
          rb[j] = packed;
          unsigned within = 0;
          for (int m = 0; m < P->NQ; ++m) {
            const unsigned v = ach[(size_t)j * P->NQ + m];
            const unsigned c = m >= 1 ? v >> 16 : 0u;
            if (c > 0 && (v & 0xffffu) != 0)
              fail(WFP_EINVAL, "stored pair-once weights: a lag's sources do not start at the row");
            acxh[(size_t)j * P->NQ + m] = make_uint2(c, within);
            within += c;
          }
          packed += within;
        }
        P->sym_rb = P->alloc<int64_t>(M);
        P->sym_acx = P->alloc<uint2>(acxh.size());
        P->sym_q = P->alloc<double>(packed + 2);
        upload(P->sym_rb, rb, s);
        upload(P->sym_acx, acxh, s);
        hipLaunchKernelGGL(k_pack_weights, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ,
                           1, ucnt_d, uoff_d, dense, uac, P->sym_rb, P->sym_q);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        P->n_weights_stored = packed;
        P->sym_upb = upb_d;
        P->sym_colpart = P->alloc<double>(np_up);
        // two sources per lane when the upper ranges are long enough to keep
        // the lanes busy (measured: faster at 206 sources per range, slower at
        // 69, where half the lanes would idle)
        P->sym_spl = np_up >= (int64_t)kSymPairedRange * M ? 2 : 1;
        // rows covering row l: j < l with up[j] > l, and j > l with up[j] > l + M
        // (periodic); up is non-decreasing, so each is a run ending at l - 1 or M - 1
        std::vector<int2> cov(M);
        {
          int64_t a = 0, b = 0;
          for (int64_t l = 0; l < M; ++l) {
            while (a < l && up[a] <= l) ++a;
            while (b < M && (int64_t)up[b] <= l + M) ++b;
            cov[l] = make_int2((int)a, periodic ? (int)std::max<int64_t>(b, l + 1) : (int)M);
          }
        }
        P->sym_cov = P->alloc<int2>(M);
        upload(P->sym_cov, cov, s);
        for (int64_t j = 0; j < M; ++j)
          P->sym_kmax = std::max(P->sym_kmax, (int)acxh[(size_t)j * P->NQ + 1].x - 1);
        P->locb = P->alloc<double>(2 * (size_t)M);
        for (void* q : {(void*)dense, (void*)uac, (void*)umlo, (void*)ust_d, (void*)ucnt_d, (void*)uoff_d,
                        (void*)ones_d})
          P->release(q);
      }
    }
    P->otf_z = P->alloc<double>(P->ngl);
    P->otf_w = P->alloc<double>(P->ngl);
    P->phitab = P->alloc<double>(tab.size());
    upload(P->otf_z, za, s);
    upload(P->otf_w, wa, s);
    // node fractions (1 + z)/2 and half weights w/2 of the symmetric kernel
    std::vector<double> nfr(P->ngl), nhw(P->ngl);
    for (int q = 0; q < P->ngl; ++q) {
      nfr[q] = 0.5 * (1.0 + za[q]);
      nhw[q] = 0.5 * wa[q];
    }
    P->otf_na = P->alloc<double>(P->ngl);
    P->otf_nw = P->alloc<double>(P->ngl);
    upload(P->otf_na, nfr, s);
    upload(P->otf_nw, nhw, s);
    upload(P->phitab, tab, s);
    P->half_beta = hb_d;
  } else {
    launch_qw((int)M, P->xs, P->nb_start, P->nb_count, P->qoff, hb_d, pbase, mlo, P->Q);
  }
  if (!P->otf) {
    unsigned long long* cnt = P->alloc<unsigned long long>(1);
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_count_nonzero, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ,
                       P->nb_count, P->qoff, P->Q, cnt);
    HIPCHK(hipGetLastError());
    unsigned long long h = 0;
    HIPCHK(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    P->n_weights_nonzero = (int64_t)h;
    // lag 1 alone (lags 0 .. 1 counted from lag 1)
    HIPCHK(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_count_nonzero, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, 2,
                       P->nb_count, P->qoff, P->Q, cnt);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    P->n_weights_lag1 = (int64_t)h;
    P->release(cnt);
  }
  // ---- pack the weights of lags >= 1 to each row's nonzero source ranges ----
  if (!P->otf) {
    for (int64_t j = 0; j < M; ++j)
      if (nbc[j] >= 65536) fail(WFP_EDOMAIN, "more than 65535 neighbours of one scatterer");
    P->ac = P->alloc<unsigned>((size_t)M * P->NQ);
    hipLaunchKernelGGL(k_row_ranges, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ,
                       P->nb_count, pbase, mlo, P->ac);
    HIPCHK(hipGetLastError());
    std::vector<unsigned> ach((size_t)M * P->NQ);
    HIPCHK(hipMemcpyAsync(ach.data(), P->ac, ach.size() * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int64_t> rb(M);
    std::vector<uint2> acxh((size_t)M * P->NQ);
    int64_t packed = 0;
    for (int64_t j = 0; j < M; ++j) {
      rb[j] = packed;
      unsigned within = 0;
      for (int m = 0; m < P->NQ; ++m) {
        const unsigned v = ach[(size_t)j * P->NQ + m];
        acxh[(size_t)j * P->NQ + m] = make_uint2(v, within);
        if (m >= 1) within += v >> 16;
      }
      packed += within;
    }
    P->nqd = (P->NQ - 1 + 3) / 4;
    P->acx = P->alloc<uint2>(acxh.size());
    upload(P->acx, acxh, s);
    HIPCHK(hipStreamSynchronize(s));
    P->n_weights_stored = packed;
    P->rowbase = P->alloc<int64_t>(M);
    P->Qc = P->alloc<double>(packed + 2);   // spare elements for paired loads
    P->locb = P->alloc<double>(2 * (size_t)M);
    // short lag blocks (few neighbours) take more lags per trip
    const double meanc = (double)packed / ((double)M * (P->NQ - 1));
    P->lgrp = meanc >= 48.0 ? 16 : (meanc >= 20.0 ? 8 : 4);
    P->lsplit = P->lgrp == 16 ? kLocalSplit : 1;
    if (P->lsplit > 1) P->locb2 = P->alloc<double>(2 * (size_t)(P->lsplit - 1) * M);
    upload(P->rowbase, rb, s);
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ, 1,
                       P->nb_count, P->qoff, P->Q, P->ac, P->rowbase, P->Qc);
    HIPCHK(hipGetLastError());
  }
  if (P->R > 0) {
    std::vector<int> rs(P->R), rc(P->R);
    std::vector<int64_t> ro(P->R);
    int64_t rt = 0;
    for (int64_t r = 0; r < P->R; ++r) {
      source_range(xs, xrh[r], P->delta, periodic, false, rs[r], rc[r]);
      ro[r] = rt;
      rt += (int64_t)rc[r] * P->NQ;
      P->n_pairs_recv += rc[r];
    }
    P->xr_h = xrh;
    P->rnbs_h = rs;
    P->rnbc_h = rc;
    P->rqoff_h = ro;
    P->xr = P->alloc<double>(P->R);
    P->rnb_start = P->alloc<int>(P->R);
    P->rnb_count = P->alloc<int>(P->R);
    P->rqoff = P->alloc<int64_t>(P->R);
    P->Qr = P->alloc<double>(rt);
    upload(P->xr, xrh, s);
    upload(P->rnb_start, rs, s);
    upload(P->rnb_count, rc, s);
    upload(P->rqoff, ro, s);
    std::vector<double> halfs(P->R, 0.5);
    double* hr_d = P->alloc<double>(P->R);
    upload(hr_d, halfs, s);
    launch_qw((int)P->R, P->xr, P->rnb_start, P->rnb_count, P->rqoff, hr_d, nullptr, nullptr, P->Qr);
    P->ri0s = P->alloc<int>(P->R);
    P->riw = P->alloc<double>((size_t)P->R * P->width);
    hipLaunchKernelGGL(k_interp_weights, dim3(nblk(P->R, 256)), dim3(256), 0, s, (int)P->R, P->nf, P->hf,
                       1.0 / P->alpha_es, P->beta_es, P->width, P->xr, P->ri0s, P->riw);
    HIPCHK(hipGetLastError());
  }
  // ---- solve: contraction bound, sweep count, tiles with halos ----
  {
    double* cr = P->alloc<double>(M);
    if (P->otf)
      hipLaunchKernelGGL(k_row_contraction, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, near_start, near_count,
                         near_off, P->Q, near_start, near_count, cr);
    else
      hipLaunchKernelGGL(k_row_contraction, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, P->nb_start,
                         P->nb_count, P->qoff, P->Q, near_start, near_count, cr);
    HIPCHK(hipGetLastError());
    std::vector<double> crh(M);
    HIPCHK(hipMemcpyAsync(crh.data(), cr, M * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    P->release(cr);
    double rho = 0;
    for (double v : crh) rho = std::max(rho, v);
    P->contraction = rho;
    if (par->solve_iters > 0) {
      P->iters = par->solve_iters;
    } else if (rho <= 0) {
      P->iters = 1;
    } else {
      if (rho >= 0.9) fail(WFP_EDOMAIN, "per-step system too weakly diagonally dominant for the Jacobi solve");
      P->iters = 1 + (int)std::ceil(std::log(1e-18) / std::log(rho));
    }
    const double reach = P->iters * P->dt * (1.0 + 1e-9) + 1e-12;
    // ---- runs of consecutive springs closer than dt: I + S is block diagonal over them ----
    std::vector<char> link(M, 0);
    for (int64_t i = 0; i < M; ++i)
      if (periodic || i + 1 < M) link[i] = pair_distance(xs[i], xs[(i + 1) % M], periodic) < P->dt;
    struct Run { int64_t start, len; };
    std::vector<Run> runs;
    bool whole_circle = false;
    {
      int64_t b0 = -1;
      if (periodic) {
        for (int64_t i = 0; i < M; ++i)
          if (!link[i]) { b0 = i; break; }
        if (b0 < 0) whole_circle = true;
      }
      if (whole_circle) {
        runs.push_back({0, M});
      } else {
        const int64_t s0 = periodic ? (b0 + 1) % M : 0;
        int64_t cur = s0, len = 1;
        for (int64_t k = 1; k < M; ++k) {
          const int64_t i = (s0 + k - 1) % M;
          if (link[i]) ++len;
          else {
            runs.push_back({cur, len});
            cur = (s0 + k) % M;
            len = 1;
          }
        }
        runs.push_back({cur, len});
      }
    }
    const int64_t kDirectMax = 96;
    // ---- direct tiles: whole small runs, contiguous, up to 256 points ----
    {
      std::vector<int> dg0, dn, dp0, pcs, pcn;
      std::vector<int64_t> pinv, gq;          // gq: weight index of each inverse-matrix coupling
      std::vector<int64_t> run_inv_off;       // per small run: offset of its inverse
      std::vector<std::array<int64_t, 2>> small;   // (start, len)
      int64_t inv_total = 0;
      int64_t next_contig = -1;
      for (const Run& r : runs) {
        if (whole_circle || r.len > kDirectMax) { next_contig = -1; continue; }
        const bool cont = (next_contig == r.start) && !dn.empty() && dn.back() + r.len <= 256;
        if (!cont) {
          dg0.push_back((int)r.start);
          dn.push_back(0);
          dp0.push_back((int)pcs.size());
        }
        const int cs = dn.back();
        for (int64_t k = 0; k < r.len; ++k) {
          pcs.push_back(cs);
          pcn.push_back((int)r.len);
          pinv.push_back(inv_total + k * r.len);
        }
        dn.back() += (int)r.len;
        run_inv_off.push_back(inv_total);
        small.push_back({r.start, r.len});
        inv_total += r.len * r.len;
        next_contig = (r.start + r.len) % M;
      }
      P->n_direct_tiles = (int)dg0.size();
      if (P->n_direct_tiles > 0) {
        // couplings inside each small run: (run, i, j) -> weight index of S_ij (lag 0)
        std::vector<int64_t> coup_q;
        std::vector<int64_t> coup_pos;   // position in the inverse-matrix buffer
        for (size_t rr = 0; rr < small.size(); ++rr) {
          const int64_t st = small[rr][0], len = small[rr][1];
          for (int64_t i = 0; i < len; ++i) {
            const int64_t gi = (st + i) % M;
            for (int64_t j = 0; j < len; ++j) {
              const int64_t gj = (st + j) % M;
              if (pair_distance(xs[gi], xs[gj], periodic) < P->dt) {
                coup_q.push_back(lag0(gi, gj));
                coup_pos.push_back(run_inv_off[rr] + i * len + j);
              }
            }
          }
        }
        int64_t* cq_d = P->alloc<int64_t>(coup_q.size());
        double* cv_d = P->alloc<double>(coup_q.size());
        upload(cq_d, coup_q, s);
        hipLaunchKernelGGL(k_gather_solve, dim3(nblk(coup_q.size(), 256)), dim3(256), 0, s,
                           (int64_t)coup_q.size(), cq_d, P->Q, cv_d, (int64_t)0, (const int64_t*)nullptr,
                           (double*)nullptr);
        HIPCHK(hipGetLastError());
        std::vector<double> cv(coup_q.size());
        HIPCHK(hipMemcpyAsync(cv.data(), cv_d, cv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        P->release(cq_d);
        P->release(cv_d);
        std::vector<double> A(inv_total, 0.0);
        for (size_t k = 0; k < coup_q.size(); ++k) A[coup_pos[k]] = cv[k];
        std::vector<double> inv(inv_total, 0.0);
        for (size_t rr = 0; rr < small.size(); ++rr) {
          const int64_t len = small[rr][1], off = run_inv_off[rr];
          for (int64_t i = 0; i < len; ++i) A[off + i * len + i] += 1.0;
          invert_dense((int)len, &A[off], &inv[off]);
        }
        P->dt_g0 = P->alloc<int>(dg0.size());
        P->dt_n = P->alloc<int>(dn.size());
        P->dt_p0 = P->alloc<int>(dp0.size());
        P->pt_cs = P->alloc<int>(pcs.size());
        P->pt_cn = P->alloc<int>(pcn.size());
        P->pt_inv = P->alloc<int64_t>(pinv.size());
        P->inv = P->alloc<double>(inv.size());
        upload(P->dt_g0, dg0, s);
        upload(P->dt_n, dn, s);
        upload(P->dt_p0, dp0, s);
        upload(P->pt_cs, pcs, s);
        upload(P->pt_cn, pcn, s);
        upload(P->pt_inv, pinv, s);
        upload(P->inv, inv, s);
      }
    }
    // ---- Jacobi tiles over the large runs: chunks of T points plus every point
    // of the same run within `reach` (a coupling never leaves its run) ----
    std::vector<int> es, el, tg0, tleft, tn;
    auto build_tiles = [&](int T) {
      es.clear(); el.clear(); tg0.clear(); tleft.clear(); tn.clear();
      int emax = 0;
      for (const Run& r : runs) {
        if (!whole_circle && r.len <= kDirectMax) continue;
        for (int64_t a0 = 0; a0 < r.len; a0 += T) {
          const int64_t b0 = std::min<int64_t>(r.len, a0 + T);
          int64_t lo = a0, hi = b0;   // run-relative, extended below
          const double xa = xs[(r.start + a0) % M], xb = xs[(r.start + b0 - 1) % M];
          if (whole_circle) {
            // circular run: extend across the wrap, at most the whole circle
            int64_t ext_l = 0, ext_r = 0;
            while (ext_l < M && pair_distance(xs[((r.start + a0 - ext_l - 1) % M + M) % M], xa, periodic) <= reach)
              ++ext_l;
            while (ext_r < M && pair_distance(xs[(r.start + b0 + ext_r) % M], xb, periodic) <= reach) ++ext_r;
            if (ext_l + ext_r + (b0 - a0) >= M) {
              lo = a0;
              hi = a0 + M;
            } else {
              lo = a0 - ext_l;
              hi = b0 + ext_r;
            }
          } else {
            while (lo > 0 && pair_distance(xs[(r.start + lo - 1) % M], xa, periodic) <= reach) --lo;
            while (hi < r.len && pair_distance(xs[(r.start + hi) % M], xb, periodic) <= reach) ++hi;
          }
          es.push_back((int)(((r.start + lo) % M + M) % M));
          el.push_back((int)(hi - lo));
          tg0.push_back((int)((r.start + a0) % M));
          tleft.push_back((int)(a0 - lo));
          tn.push_back((int)(b0 - a0));
          emax = std::max(emax, (int)(hi - lo));
        }
      }
      return emax;
    };
    int T = 64, emax = build_tiles(T);
    while (emax > 4 * T && T < 2048) {
      T *= 2;
      emax = build_tiles(T);
    }
    P->T = T;
    P->ntile = (int)es.size();
    P->ext_max = emax;
    P->solve_threads = (int)std::min<int64_t>(256, 64 * nblk(std::max(emax, 1), 64));
    {
      // LDS the tiles would need: four vectors plus the tile's CSR
      size_t need = 0;
      for (int t = 0; t < P->ntile; ++t) {
        int64_t ne = 0;
        for (int e = 0; e < el[t]; ++e) ne += nc[((int64_t)es[t] + e) % M];
        need = std::max(need, (size_t)emax * 4 * sizeof(double) + (size_t)ne * (sizeof(double) + sizeof(int)) +
                                  (size_t)(emax + 1) * sizeof(int));
      }
      P->solve_global = need > 160 * 1024;
    }
    if (P->solve_global) {
      // every row by global sweeps; the direct and tiled paths are not used
      P->n_direct_tiles = 0;
      P->ntile = 0;
      std::vector<int> gp(M + 1, 0), gc;
      std::vector<int64_t> geq, grq(M);
      for (int64_t g = 0; g < M; ++g) {
        grq[g] = lag0(g, g);
        for (int k = 0; k < nc[g]; ++k) {
          const int64_t l = (ns[g] + k) % M;
          if (l == g) continue;
          gc.push_back((int)l);
          geq.push_back(lag0(g, l));
        }
        gp[g + 1] = (int)gc.size();
      }
      // a wavefront per row when rows are long
      P->g_wave = gc.size() > (size_t)16 * M;
      P->g_ptr = P->alloc<int>(M + 1);
      P->g_col = P->alloc<int>(gc.size());
      P->g_val = P->alloc<double>(gc.size());
      P->g_dinv = P->alloc<double>(M);
      P->g_rhs = P->alloc<double>(M);
      P->g_xa = P->alloc<double>(M);
      P->g_xb = P->alloc<double>(M);
      upload(P->g_ptr, gp, s);
      upload(P->g_col, gc, s);
      int64_t* eq_d = P->alloc<int64_t>(geq.size());
      int64_t* rq_d = P->alloc<int64_t>(M);
      upload(eq_d, geq, s);
      upload(rq_d, grq, s);
      hipLaunchKernelGGL(k_gather_solve, dim3(nblk(std::max<int64_t>((int64_t)geq.size(), M), 256)), dim3(256), 0,
                         s, (int64_t)geq.size(), eq_d, P->Q, P->g_val, (int64_t)M, rq_d, P->g_dinv);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      P->release(eq_d);
      P->release(rq_d);
    }
    if (P->ntile > 0) {
      std::vector<int> tr0(P->ntile), rg, rptr, col;
      std::vector<int64_t> rq, eq;
      rptr.push_back(0);
      for (int t = 0; t < P->ntile; ++t) {
        tr0[t] = (int)rg.size();
        for (int e = 0; e < el[t]; ++e) {
          const int64_t g = ((int64_t)es[t] + e) % M;
          rg.push_back((int)g);
          rq.push_back(lag0(g, g));
          for (int k = 0; k < nc[g]; ++k) {
            const int64_t l = (ns[g] + k) % M;
            if (l == g) continue;
            const int64_t le = (l - es[t] + M) % M;
            if (le >= el[t]) continue;   // outside the halo: only reaches rows that are not kept
            col.push_back((int)le);
            eq.push_back(lag0(g, l));
          }
          rptr.push_back((int)col.size());
        }
      }
      P->tile_r0 = P->alloc<int>(P->ntile);
      P->tile_el = P->alloc<int>(P->ntile);
      P->tile_g0 = P->alloc<int>(P->ntile);
      P->tile_left = P->alloc<int>(P->ntile);
      P->tile_n = P->alloc<int>(P->ntile);
      P->srow_g = P->alloc<int>(rg.size());
      P->srow_ptr = P->alloc<int>(rptr.size());
      P->scol = P->alloc<int>(col.size());
      P->srow_dinv = P->alloc<double>(rg.size());
      P->sval = P->alloc<double>(col.size());
      upload(P->tile_r0, tr0, s);
      upload(P->tile_el, el, s);
      upload(P->tile_g0, tg0, s);
      upload(P->tile_left, tleft, s);
      upload(P->tile_n, tn, s);
      upload(P->srow_g, rg, s);
      upload(P->srow_ptr, rptr, s);
      upload(P->scol, col, s);
      int64_t* eq_d = P->alloc<int64_t>(eq.size());
      int64_t* rq_d = P->alloc<int64_t>(rq.size());
      upload(eq_d, eq, s);
      upload(rq_d, rq, s);
      const int64_t ne = (int64_t)col.size(), nr = (int64_t)rg.size();
      int max_ne = 0;
      for (int t = 0; t < P->ntile; ++t) max_ne = std::max(max_ne, rptr[tr0[t] + el[t]] - rptr[tr0[t]]);
      P->lds_jac = (size_t)emax * 4 * sizeof(double) + (size_t)max_ne * (sizeof(double) + sizeof(int)) +
                   (size_t)(emax + 1) * sizeof(int);
      if (P->lds_jac > 160 * 1024) fail(WFP_EDOMAIN, "solve tile too large for one workgroup");
      hipLaunchKernelGGL(k_gather_solve, dim3(nblk(std::max(ne, nr), 256)), dim3(256), 0, s, ne, eq_d, P->Q,
                         P->sval, nr, rq_d, P->srow_dinv);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(s));
      P->release(eq_d);
      P->release(rq_d);
    }
  }
  // the dense weights of the scatterer rows are no longer needed
  HIPCHK(hipStreamSynchronize(s));
  P->release(P->Q);
  P->Q = nullptr;
  if (mlo) P->release(mlo);
  P->release(pbase);
  P->release(near_start);
  P->release(near_count);
  P->release(near_off);
  P->ginc = P->alloc<double>(M);
  P->loc = P->alloc<double>(M);
  if (!periodic) {
    P->tw_rbc = P->alloc<double2>(2 * P->K);
    std::vector<double2> tw(2 * P->K);
    for (int64_t t = 0; t < 2 * P->K; ++t) {
      const long double a = -3.14159265358979323846264338327950288L * (long double)t / (long double)P->K;
      tw[t] = make_double2((double)std::cos(a), (double)std::sin(a));
    }
    upload(P->tw_rbc, tw, s);
    P->rbc_u = P->alloc<double>(2 * P->K);
    P->rbc_v = P->alloc<double>(2 * P->K);
    if (P->rbc_split) {
      P->rbc_z = P->alloc<double2>(2 * P->K);
      P->rbc_t = P->alloc<double2>(2 * P->K);
    }
  }
  // kernels with more than 64 KB of LDS
  HIPCHK(hipFuncSetAttribute((const void*)k_rbc_to_grid, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_rbc_fft_pass1, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_rbc_fft_pass2, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_hist_a, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_hist_c, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_hist_a_wide, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_hist_c_wide, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_rbc_to_modes, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_solve, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)k_hist_b, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  if (P->otf) {
    const size_t sym_lds = (size_t)(P->NQ + kOtfRows) * kOtfChunk * sizeof(double) +
                           (size_t)kPhiPieces * (kPhiDeg + 1) * sizeof(double) +
                           (size_t)kOtfRows * (kMaxOtfLags + 1) * sizeof(double) + 128 * sizeof(double);
    if (P->NQ - 1 > kMaxOtfLags || sym_lds > 160 * 1024)
      fail(WFP_EDOMAIN, "on-the-fly local sum: too many lags for the LDS stage");
    const void* sfns[6] = {(const void*)k_local_otf_sym<2>, (const void*)k_local_otf_sym<4>,
                           (const void*)k_local_otf_sym<6>, (const void*)k_local_otf_sym<8>,
                           (const void*)k_local_otf_sym<10>, (const void*)k_local_otf_sym<12>};
    const int sdyn = (int)((size_t)(P->NQ + kOtfRows) * kOtfChunk * sizeof(double));
    for (const void* f : sfns) HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, sdyn));
  }
  // the column pass holds 6 n1 complex values and the FIR partial sums of G
  // tap groups ([G][2 n1] double4); column pairs of 400 modes or more keep one
  // or two modes per thread with G = 2 (and fit two blocks per compute unit),
  // shorter ones split the taps 8 ways to give every thread work
  P->fir_groups = 2 * P->n1 >= 400 ? 2 : 8;
  P->lds_b = 6 * (size_t)P->n1 * sizeof(double2) + (size_t)P->fir_groups * 2 * P->n1 * sizeof(double4);
  if (P->lds_b > 160 * 1024) fail(WFP_EDOMAIN, "four-step factor n1 too long for the history kernel's LDS");
  {
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, P->device));
    const int ncu = prop.multiProcessorCount;
    if (P->overlap_cus == 0) {
      // the chain on one XCD (its own L2) while the local sum streams its
      // weights on the others, when the local sum is long enough to hide it
      int nx = 1;
      if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, P->device) != hipSuccess || nx < 2) nx = 1;
      const bool worth = 8.0 * (double)P->n_weights_stored >= 64.0 * 1024 * 1024;
      P->overlap_cus = (nx > 1 && worth) ? ncu / nx : -1;
    }
  }
  if (P->overlap_cus > 0) set_overlap(P, P->overlap_cus);
  zero_state(P);
  HIPCHK(hipStreamSynchronize(s));
}

// Local sum of lags >= 1 with the weights evaluated on the fly, scaled per row:
// each unordered pair once (k_local_otf_sym), then the per-row totals
// (k_local_otf_reduce).  ea / eb bracket both launches.
// The on-the-fly schedule (the whole local sum after the previous level's
// solve); stored weights, per ordered pair or once per pair, take the
// pipelined one (lags >= 2 ahead, lag 1 after the previous solve).
bool otf_schedule(const wfp_plan* P) { return P->otf && !P->sym_stored; }

void launch_local_otf(wfp_plan* P, hipStream_t s, const double* hist, int64_t L, const double* scale, double* out,
                      hipEvent_t ea = nullptr, hipEvent_t eb = nullptr) {
  const int nblocks = 8 * (int)nblk(P->otf_nblk, 8);
  const int periodic = P->boundary == WFP_PERIODIC ? 1 : 0;
  const size_t lds = (size_t)(P->NQ + kOtfRows) * kOtfChunk * sizeof(double);
#define WFP_OTF(PP)                                                                                               \
  hipExtLaunchKernelGGL(k_local_otf_sym<PP>, dim3(nblocks), dim3(64 * kOtfRows), lds, s, ea, nullptr, 0,          \
                        (int)P->M, P->NH, P->NQ, L, P->otf_up_end, P->otf_blk_end, P->otf_part_off, P->otf_nblk,  \
                        P->xs, hist, periodic, P->dt, P->delta, P->W, P->ngl, P->otf_na, P->otf_nw, P->phitab,  \
                        P->otf_rowacc, P->otf_part)
  if (P->sym_stored) {
    hipExtLaunchKernelGGL(P->sym_spl == 2 ? k_local_sym_rows<2> : k_local_sym_rows<1>,
                          dim3(8 * nblk(nblk(P->M, 4), 8)), dim3(256), 0, s, ea, nullptr, 0,
                          (int)P->M, P->NH, P->NQ, L, 1, P->otf_up_end, hist, P->sym_rb, P->sym_acx, P->sym_q,
                          P->sym_upb, P->otf_rowacc, P->sym_colpart);
    hipExtLaunchKernelGGL(k_local_sym_reduce, dim3(nblk(P->M, 64)), dim3(64 * kReduceWaves), 0, s, nullptr, eb, 0, (int)P->M,
                          P->sym_cov, P->sym_upb, P->otf_rowacc, P->sym_colpart, scale, out);
    return;
  }
  switch (P->p) {
    case 2: WFP_OTF(2); break;
    case 4: WFP_OTF(4); break;
    case 6: WFP_OTF(6); break;
    case 8: WFP_OTF(8); break;
    case 10: WFP_OTF(10); break;
    default: WFP_OTF(12); break;
  }
#undef WFP_OTF
  hipExtLaunchKernelGGL(k_local_otf_reduce, dim3(nblk(P->M, 256)), dim3(256), 0, s, nullptr, eb, 0, (int)P->M,
                        P->otf_nblk, periodic, P->otf_blk_end, P->otf_part_off, P->otf_rowacc, P->otf_part, scale,
                        out);
}

// The march state a level reads and updates: density history ring, spectra
// ring, alpha, alpha'.  The plan's own state, the replay copy and the adjoint
// state of the gradient pass all use the same level code.
struct StateRef {
  double* hist;
  double2* ring;
  double2* alpha;
  double2* dalpha;
};

StateRef main_state(wfp_plan* P) { return {P->hist, P->ring, P->alpha, P->dalpha}; }

// Row passes of the fine-grid transform, at the plan's block size.
void launch_hist_a(wfp_plan* P, hipStream_t s, const double* sig, ExtraSources ex) {
  const size_t lds = P->n2 * sizeof(double2);
  if (P->hist_threads == 256)
    hipLaunchKernelGGL(k_hist_a, dim3(P->n1), dim3(256), lds, s, P->fft_n2, P->n1, sig, (int)P->M, P->cstart,
                       P->ccount, P->swoff, P->sw, P->tw, P->T1, ex);
  else {
    hipLaunchKernelGGL(k_spread_grid, dim3(nblk(P->nf, 256)), dim3(256), 0, s, P->nf, sig, (int)P->M, P->cstart,
                       P->ccount, P->swoff, P->sw, ex, P->gsp);
    hipLaunchKernelGGL(k_hist_a_wide, dim3(8 * nblk(P->n1, 8)), dim3(1024), lds, s, P->fft_n2, P->n1, P->gsp, P->tw,
                       P->T1);
  }
}

void launch_hist_c(wfp_plan* P, hipStream_t s, double2* grid) {
  const size_t lds = P->n2 * sizeof(double2);
  if (P->hist_threads == 256)
    hipLaunchKernelGGL(k_hist_c, dim3(P->n1), dim3(256), lds, s, P->fft_n2, P->n1, P->V, P->tw, grid);
  else
    hipLaunchKernelGGL(k_hist_c_wide, dim3(8 * nblk(P->n1, 8)), dim3(1024), lds, s, P->fft_n2, P->n1, P->V, P->tw,
                       grid);
}

// Stored weights: the lags >= 2 part of level L's local sum into locb[L & 1]
// (reads sigma^{L-2} and older only), and its lag-1 part added to it.
// The stored-weight local sum of lags m0 <= m < NQ into out, with the plan's
// lanes per lag.
// out2 != NULL (16 lanes per lag only): P->lsplit wavefronts per row, parts
// 1 .. lsplit - 1 of the lags into out2 (M values each).
void launch_local_sum(wfp_plan* P, hipStream_t s, const double* hist, int64_t L, int m0, double* out,
                      hipEvent_t ea = nullptr, hipEvent_t eb = nullptr, double* out2 = nullptr) {
  const int nsplit = out2 ? P->lsplit : 1;
  const int64_t waves = nsplit * P->M;
  const int nb = 8 * (int)nblk(nblk(waves, kRowThreads / 64), 8);
#define WFP_LOC(KER)                                                                                             \
  hipExtLaunchKernelGGL(KER, dim3(nb), dim3(kRowThreads), 0, s, ea, eb, 0, (int)P->M, P->NQ, P->NH, L, m0, P->NQ, \
                        P->nb_start, P->rowbase, P->acx, P->Qc, hist, (const double*)nullptr, out)
  switch (P->lgrp) {
    case 8: WFP_LOC(k_local_rhs_g8); break;
    case 4: WFP_LOC(k_local_rhs_g4); break;
    default:
      hipExtLaunchKernelGGL(k_local_rhs, dim3(nb), dim3(kRowThreads), 0, s, ea, eb, 0, (int)P->M, P->NQ, P->NH, L,
                            m0, P->NQ, P->nb_start, P->rowbase, P->acx, P->Qc, hist, (const double*)nullptr, out,
                            out2, nsplit);
      break;
  }
#undef WFP_LOC
}

// The lags >= 2 part of level L's local sum: rows of 16 lanes per lag split
// over P->lsplit wavefronts (part 0 into locb, the others into locb2, all
// summed by the lag-1 part).
double* locb_second(wfp_plan* P, int64_t L) {
  return P->lsplit > 1 ? P->locb2 + (L & 1) * (P->lsplit - 1) * P->M : nullptr;
}

void launch_local_big(wfp_plan* P, hipStream_t s, const double* hist, int64_t L, hipEvent_t ea = nullptr,
                      hipEvent_t eb = nullptr) {
  if (P->sym_stored) {
    hipExtLaunchKernelGGL(P->sym_spl == 2 ? k_local_sym_rows<2> : k_local_sym_rows<1>,
                          dim3(8 * nblk(nblk(P->M, 4), 8)), dim3(256), 0, s, ea, nullptr, 0,
                          (int)P->M, P->NH, P->NQ, L, 2, P->otf_up_end, hist, P->sym_rb, P->sym_acx, P->sym_q,
                          P->sym_upb, P->otf_rowacc, P->sym_colpart);
    hipExtLaunchKernelGGL(k_local_sym_reduce, dim3(nblk(P->M, 64)), dim3(64 * kReduceWaves), 0, s, nullptr, eb, 0, (int)P->M,
                          P->sym_cov, P->sym_upb, P->otf_rowacc, P->sym_colpart, P->half_beta,
                          P->locb + (L & 1) * P->M);
    return;
  }
  launch_local_sum(P, s, hist, L, 2, P->locb + (L & 1) * P->M, ea, eb, locb_second(P, L));
}

// Row of level L's driving data g_j(t_L) (eq. (gj)).  The values depend on L
// only, so they are computed for g_chunk levels at a time, on `s` (every
// reader of the previous chunk is ordered before it on that stream, or
// before the solve the stream has waited for).
const double* driving_row(wfp_plan* P, hipStream_t s, int64_t L) {
  double* buf = P->g_ext;
  int chunk = P->g_ext_chunk;
  if (!buf) {
    if (!P->gbuf) {
      P->g_chunk = (int)std::max<int64_t>(1, std::min<int64_t>(256, (int64_t)(8 << 20) / P->M));
      P->gbuf = P->alloc<double>((size_t)P->g_chunk * P->M);
    }
    buf = P->gbuf;
    chunk = P->g_chunk;
  }
  if (P->g_lvl0 < 0 || L < P->g_lvl0 || L >= P->g_lvl0 + chunk) {
    const Packets pk{P->npk, P->boundary == WFP_PERIODIC ? 1 : 0, P->packets};
    int pp = 1;
    while (pp < P->npk) pp *= 2;
    hipLaunchKernelGGL(k_incident_levels, dim3(nblk(P->M, 256 / pp), chunk), dim3(256), 0, s, (int)P->M, L,
                       P->dt, P->xs, P->beta, pk, pp, buf);
    P->g_lvl0 = L;
  }
  return buf + (L - P->g_lvl0) * P->M;
}

void launch_local_lag1(wfp_plan* P, hipStream_t s, const double* hist, int64_t L) {
  if (P->sym_stored) {
    hipLaunchKernelGGL(k_local_sym_lag1, dim3(nblk(P->M, 16)), dim3(256), 0, s, (int)P->M, P->NQ, P->NH, L,
                       P->boundary == WFP_PERIODIC ? 1 : 0, P->sym_kmax, P->sym_rb, P->sym_acx, P->sym_q, hist,
                       P->half_beta, P->locb + (L & 1) * P->M, P->loc);
    return;
  }
  const int nb = 8 * (int)nblk(nblk(P->M, 16), 8);   // 16 rows per block of 256 threads
  hipLaunchKernelGGL(k_local_lag1, dim3(nb), dim3(kRowThreads), 0, s, (int)P->M, P->NQ, P->NH, L, P->nb_start,
                     P->rowbase, P->acx, P->Qc, hist, P->locb + (L & 1) * P->M, locb_second(P, L), P->lsplit - 1,
                     P->loc);
}

// One level L, in stream order: driving data (unless `driven`: P->ginc already
// holds it), local sum (levels < L), the history part (three kernels; the
// free-space projection when due), solve, receivers.  Stored weights: the
// local sum is its lags >= 2 part and its lag-1 part.  `ahead`: the driving
// data and the whole local sum of level L were launched on P->sd by the
// caller, which signals ev_big[L & 1] after them.
void march_level(wfp_plan* P, const StateRef& S, int64_t L, bool driven, const ExtraSources& ex, double* save,
                 double* u_recv_row, bool overlap = false, bool ahead = false, const double* local_ready = nullptr) {
  // overlap: the history chain on P->sb (its own compute units) after the
  // previous level's solve and receivers, everything else on P->sa; the solve
  // waits for both.  ahead: the solve and receivers follow the chain on P->sb
  // (no wait between queues on the chain -> solve -> chain path).
  // local_ready: the level's explicit local sum, already formed (copied in
  // place of the local-sum kernels).
  hipStream_t sc = overlap ? P->sb : P->stream;
  hipStream_t s = overlap ? (ahead ? P->sb : P->sa) : P->stream;
  if (overlap && sc != s) HIPCHK(hipStreamWaitEvent(sc, P->ev_solved, 0));
  const bool periodic = P->boundary == WFP_PERIODIC;
  const unsigned nb_b = (unsigned)(P->n2 / 2 + 1);
  const size_t lds_b = P->lds_b;
  const double* sig_prev = S.hist + (int64_t)(((L - 1) % P->NH + P->NH) % P->NH) * P->M;
  const double* gin = driven ? P->ginc : driving_row(P, s, L);
  {
    // timed with events bound to the kernel's own dispatch (no marker gaps)
    hipEvent_t ea = nullptr, eb = nullptr;
    const bool timed = P->profiling && !local_ready;
    if (timed) {
      ea = take_event(P);
      eb = take_event(P);
    }
    if (local_ready) {
      HIPCHK(hipMemcpyAsync(P->loc, local_ready, P->M * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else if (otf_schedule(P) && overlap) {
      // on the local sum's compute units, joined before the solve
      HIPCHK(hipStreamWaitEvent(P->sd, P->ev_solved, 0));
      launch_local_otf(P, P->sd, S.hist, L, P->half_beta, P->loc);
      HIPCHK(hipEventRecord(P->ev_big[L & 1], P->sd));
      HIPCHK(hipStreamWaitEvent(s, P->ev_big[L & 1], 0));
    } else if (otf_schedule(P)) {
      launch_local_otf(P, s, S.hist, L, P->half_beta, P->loc, ea, eb);
    } else if (!ahead) {
      launch_local_big(P, s, S.hist, L, ea, eb);
    }
    if (timed) {
      P->pending.push_back({WFP_STAGE_LOCAL, ea, eb});
      if (P->pending.size() >= 1024) flush_profile(P);
    }
  }
  {
    StageTimer st(P, WFP_STAGE_SPREAD, sc);
    launch_hist_a(P, sc, sig_prev, ex);
  }
  const bool rbc = !periodic && L > 0 && L % P->rbc_period == 0;
  {
    StageTimer st(P, WFP_STAGE_MODES, sc);
    hipLaunchKernelGGL(k_hist_b, dim3(nb_b), dim3(512), lds_b, sc, rbc ? 1 : 0, P->fft_n1, P->n2, P->K, P->W, L,
                       P->npos, P->T1, P->tw, P->tw1, P->dk1, P->dk2, P->pk, P->qk, P->rot, S.ring, S.alpha,
                       S.dalpha, P->ybuf, P->V, P->fir_groups, P->hist_threads == 1024 ? 1 : 0);
  }
  if (rbc) {
    StageTimer st(P, WFP_STAGE_RBC, sc);
    if (!P->rbc_split) {
      hipLaunchKernelGGL(k_rbc_to_grid, dim3(2), dim3(kFftThreads), P->lds_rbc, sc, P->fft_rbc, P->K, P->n1,
                         P->n2, S.alpha, S.dalpha, P->tw_rbc, (double2*)P->rbc_u, (double2*)P->rbc_v);
      hipLaunchKernelGGL(k_rbc_to_modes, dim3(2), dim3(kFftThreads), P->lds_rbc, sc, P->fft_rbc, P->K, P->n1,
                         P->n2, P->W, P->h_rbc, P->delta_s, P->cheb_phi, P->cheb_g, P->ncheb, P->rbc_u, P->rbc_v,
                         P->tw_rbc, P->dk2, S.alpha, S.dalpha, P->ybuf);
    } else {
      const unsigned ne = (unsigned)nblk(2 * P->K, 256);
      const dim3 g1(P->rbc_a, 2), g2(P->rbc_b, 2);
      const size_t l1 = P->rbc_b * sizeof(double2), l2 = P->rbc_a * sizeof(double2);
      hipLaunchKernelGGL(k_rbc_grid_pack, dim3(ne), dim3(256), 0, sc, P->K, P->n1, P->n2, S.alpha, S.dalpha,
                         P->tw_rbc, P->rbc_z);
      hipLaunchKernelGGL(k_rbc_fft_pass1, g1, dim3(256), l1, sc, P->fft_rbc_b, P->rbc_a, P->K, P->tw_rbc,
                         P->rbc_z, P->rbc_t);
      hipLaunchKernelGGL(k_rbc_fft_pass2, g2, dim3(256), l2, sc, P->fft_rbc_a, P->rbc_b, P->K, P->tw_rbc,
                         P->rbc_t, (double2*)P->rbc_u, (double2*)P->rbc_v, 1);
      hipLaunchKernelGGL(k_rbc_modes_pack, dim3(ne), dim3(256), 0, sc, P->K, P->W, P->h_rbc, P->delta_s,
                         P->cheb_phi, P->cheb_g, P->ncheb, P->rbc_u, P->rbc_v, P->rbc_z);
      hipLaunchKernelGGL(k_rbc_fft_pass1, g1, dim3(256), l1, sc, P->fft_rbc_b, P->rbc_a, P->K, P->tw_rbc,
                         P->rbc_z, P->rbc_t);
      hipLaunchKernelGGL(k_rbc_fft_pass2, g2, dim3(256), l2, sc, P->fft_rbc_a, P->rbc_b, P->K, P->tw_rbc,
                         P->rbc_t, P->rbc_z, P->rbc_z + P->K, 0);
      hipLaunchKernelGGL(k_rbc_modes_unpack, dim3((unsigned)nblk(2 * (P->K + 1), 256)), dim3(256), 0, sc, P->K,
                         P->n1, P->n2, P->rbc_z, P->tw_rbc, P->dk2, S.alpha, S.dalpha, P->ybuf);
    }
    hipLaunchKernelGGL(k_hist_b, dim3(nb_b), dim3(512), lds_b, sc, 2, P->fft_n1, P->n2, P->K, P->W, L, P->npos,
                       P->T1, P->tw, P->tw1, P->dk1, P->dk2, P->pk, P->qk, P->rot, S.ring, S.alpha, S.dalpha,
                       P->ybuf, P->V, P->fir_groups, P->hist_threads == 1024 ? 1 : 0);
  }
  {
    StageTimer st(P, WFP_STAGE_FFT_INV, sc);
    launch_hist_c(P, sc, (double2*)P->grid2);
  }
  if (overlap && sc != s) {
    HIPCHK(hipEventRecord(P->ev_chain, sc));
    HIPCHK(hipStreamWaitEvent(s, P->ev_chain, 0));
  }
  double* slot = S.hist + (int64_t)(L % P->NH) * P->M;
  {
    StageTimer st(P, WFP_STAGE_SOLVE, s);
    if (ahead) HIPCHK(hipStreamWaitEvent(s, P->ev_big[L & 1], 0));   // driving data and local sum of level L
    else if (!otf_schedule(P)) launch_local_lag1(P, s, S.hist, L);
    if (P->n_direct_tiles > 0)
      hipLaunchKernelGGL(k_solve_direct, dim3(P->n_direct_tiles), dim3(256), 0, s, (int)P->M, P->dt_g0, P->dt_n,
                         P->dt_p0, P->pt_cs, P->pt_cn, P->pt_inv, P->inv, gin, P->loc, P->i0s, P->iw,
                         P->beta, P->grid2, P->nf, P->width, slot, save, P->perm);
    if (P->ntile > 0)
      hipLaunchKernelGGL(k_solve, dim3(P->ntile), dim3(P->solve_threads), P->lds_jac, s, (int)P->M, P->iters,
                         P->ext_max, P->tile_r0, P->tile_el, P->tile_g0, P->tile_left, P->tile_n, P->srow_g,
                         P->srow_dinv, P->srow_ptr, P->scol, P->sval, gin, P->loc, P->i0s, P->iw, P->beta,
                         P->grid2, P->nf, P->width, slot, save, P->perm);
    if (P->solve_global) {
      const unsigned nb = nblk(P->M, 256);
      double* xa = P->g_xa;
      double* xb = P->g_xb;
      hipLaunchKernelGGL(k_solve_rhs, dim3(nb), dim3(256), 0, s, (int)P->M, gin, P->loc, P->beta, P->i0s, P->iw,
                         P->grid2, P->nf, P->width, P->g_dinv, P->g_rhs, P->iters > 1 ? xa : slot);
      if (P->iters == 1 && save)
        hipLaunchKernelGGL(k_unsort, dim3(nb), dim3(256), 0, s, (int)P->M, P->perm, slot, save);
      for (int it = 1; it < P->iters; ++it) {
        const bool last = it == P->iters - 1;
        double* out = last ? slot : xb;
        if (P->g_wave)
          hipLaunchKernelGGL(k_jacobi_sweep_wave, dim3(nblk(P->M, 4)), dim3(256), 0, s, (int)P->M, P->g_ptr,
                             P->g_col, P->g_val, P->g_dinv, P->g_rhs, xa, out, last ? save : nullptr, P->perm);
        else
          hipLaunchKernelGGL(k_jacobi_sweep, dim3(nb), dim3(256), 0, s, (int)P->M, P->g_ptr, P->g_col, P->g_val,
                             P->g_dinv, P->g_rhs, xa, out, last ? save : nullptr, P->perm);
        std::swap(xa, xb);
      }
    }
  }
  if (P->R > 0 && u_recv_row) {
    StageTimer st(P, WFP_STAGE_RECV, s);
    hipLaunchKernelGGL(k_receivers, dim3(P->R), dim3(1024), 0, s, (int)P->M, P->NQ, P->NH, L, P->rnb_start,
                       P->rnb_count, P->rqoff, P->Qr, S.hist, P->ri0s, P->riw, P->grid2, P->nf, P->width,
                       u_recv_row);
  }
  // the next level's chain overwrites grid2, read by the solve and receivers above
  if (overlap) HIPCHK(hipEventRecord(P->ev_solved, s));
}

size_t state_bytes(const wfp_plan* P) {
  return (size_t)P->NH * P->M * sizeof(double) + ((size_t)P->W + 2) * P->npos * sizeof(double2);
}

// Copy a whole state (hist, ring, alpha, alpha') to or from a flat buffer.
void copy_state(wfp_plan* P, const StateRef& S, char* buf, bool to_buf) {
  hipStream_t s = P->stream;
  const size_t nh = (size_t)P->NH * P->M * sizeof(double), nr = (size_t)P->W * P->npos * sizeof(double2),
               na = (size_t)P->npos * sizeof(double2);
  char* parts[4] = {(char*)S.hist, (char*)S.ring, (char*)S.alpha, (char*)S.dalpha};
  const size_t sizes[4] = {nh, nr, na, na};
  size_t off = 0;
  for (int i = 0; i < 4; ++i) {
    if (to_buf) HIPCHK(hipMemcpyAsync(buf + off, parts[i], sizes[i], hipMemcpyDeviceToDevice, s));
    else HIPCHK(hipMemcpyAsync(parts[i], buf + off, sizes[i], hipMemcpyDeviceToDevice, s));
    off += sizes[i];
  }
}

void zero_state_ref(wfp_plan* P, const StateRef& S) {
  auto fill = [&](double* ptr, int64_t n) {
    hipLaunchKernelGGL(k_fill, dim3(nblk(n, 256)), dim3(256), 0, P->stream, ptr, n, 0.0);
  };
  fill(S.hist, (int64_t)P->NH * P->M);
  fill((double*)S.ring, 2 * (int64_t)P->W * P->npos);
  fill((double*)S.alpha, 2 * P->npos);
  fill((double*)S.dalpha, 2 * P->npos);
  HIPCHK(hipGetLastError());
}

void dterm_setup(wfp_plan* P);
void fwd_dterm(wfp_plan* P, const StateRef& S, int64_t L, double* out);

void run_levels(wfp_plan* P, int64_t n, double* sigma_out, int64_t save_every, double* u_recv_out) {
  const StateRef S = main_state(P);
  const ExtraSources none{nullptr, 0, nullptr, nullptr, nullptr, nullptr};
  // recording: every level's densities and forward derivative term, for a
  // gradient pass without the forward replay
  const bool rec = P->ckpt_every < 0 && P->ck_from0;
  const int64_t RC = -(int64_t)P->ckpt_every, hd = P->NQ - 1;
  if (rec && n > 0) dterm_setup(P);
  // the concurrent chain is used when configured and no checkpoints are taken
  // (per-stage timing measures each stage alone: one stream while profiling)
  const bool ov = P->overlap_cus > 0 && P->ckpt_every == 0 && n > 0 && !P->profiling;
  // stored weights, concurrent chain: once level L - 1 is solved, sd computes
  // level L's driving data and lag-1 part, then the lags >= 2 part of level
  // L + 1 (it needs sigma^{L-1} and older only), while sb runs level L's chain
  // and sa its solve
  const bool ahead = ov && !otf_schedule(P);
  // the queue that solves (and signals ev_solved)
  hipStream_t sm = ahead ? P->sb : P->sa;
  if (ov) {
    // order after earlier work on the caller's stream
    HIPCHK(hipEventRecord(P->ev_join, P->stream));
    HIPCHK(hipStreamWaitEvent(sm, P->ev_join, 0));
    HIPCHK(hipEventRecord(P->ev_solved, sm));
  }
  if (ahead) {
    HIPCHK(hipStreamWaitEvent(P->sd, P->ev_solved, 0));
    launch_local_big(P, P->sd, S.hist, P->level);
  }
  for (int64_t i = 0; i < n; ++i) {
    const int64_t L = P->level + i;
    if (ahead) {
      // sigma^{L-1} and older are final once level L - 1 is solved
      HIPCHK(hipStreamWaitEvent(P->sd, P->ev_solved, 0));
      driving_row(P, P->sd, L);
      launch_local_lag1(P, P->sd, S.hist, L);
      HIPCHK(hipEventRecord(P->ev_big[L & 1], P->sd));
      if (i + 1 < n) launch_local_big(P, P->sd, S.hist, L + 1);
    }
    if (P->ckpt_every > 0 && P->ck_from0 && L > 0 && L % P->ckpt_every == 0) {
      const size_t c = (size_t)(L / P->ckpt_every) - 1;
      while (P->ckpts.size() <= c) P->ckpts.push_back(P->alloc<char>(state_bytes(P)));
      copy_state(P, S, P->ckpts[c], true);
    }
    const size_t rb = rec ? (size_t)(L / RC) : 0;
    if (rec && L % RC == 0) {
      while (P->rec_D.size() <= rb) {
        double* sig = P->alloc<double>((size_t)(RC + hd) * P->M);
        double* dt = P->alloc<double>((size_t)RC * P->M);
        P->rec_sig.push_back(sig);
        P->rec_D.push_back(dt);
      }
      if (hd > 0)
        hipLaunchKernelGGL(k_seg_head, dim3(nblk(hd * P->M, 256)), dim3(256), 0, P->stream, (int)P->M, P->NH, L,
                           (int)hd, S.hist, P->rec_sig[rb]);
    }
    double* save = (sigma_out && i % save_every == 0) ? sigma_out + (i / save_every) * P->M : nullptr;
    march_level(P, S, L, false, none, save, u_recv_out ? u_recv_out + i * P->R : nullptr, ov, ahead);
    if (rec) {
      const int64_t r = L - (int64_t)rb * RC;
      HIPCHK(hipMemcpyAsync(P->rec_sig[rb] + (hd + r) * P->M, S.hist + (L % P->NH) * P->M, P->M * sizeof(double),
                            hipMemcpyDeviceToDevice, P->stream));
      fwd_dterm(P, S, L, P->rec_D[rb] + r * P->M);
    }
  }
  if (ov) {
    // later work on the caller's stream waits for the whole run
    HIPCHK(hipEventRecord(P->ev_join, sm));
    HIPCHK(hipStreamWaitEvent(P->stream, P->ev_join, 0));
  }
  HIPCHK(hipGetLastError());
  P->level += n;
}

// ---- gradient pass -------------------------------------------------------
// The loss J depends on the receiver values u_r^L, L = 0..N-1, and the caller
// passes e = dJ/du.  Transposing the level (eqs. (periodicIE_disc),
// (hkcompdisc), (densco), (historySol1)) gives the same level run backwards in
// time: with q^L = -beta lambda^L (lambda the adjoint of sigma^L),
//   (I + S) q^L = -beta (sum_r sum_{m>=0} (1/2) Q_m(d_r.) e_r^{L+m}
//                        + sum_{m>=1} (1/2) Q_m q^{L+m} + u_H^adj),
// where u_H^adj is the history field of the sources q (scatterers) and e
// (receivers) at the later levels, computed by the forward history kernels on
// a second state whose level counter runs N-1-L.  Then
//   dJ/dbeta_j = -sum_L q_j^L sigma_j^L / beta_j^2,
//   dJ/dx_j    =  sum_L [ q_j^L D_j^L + sigma_j^L Dadj_j^L ],
// D = f'(x_j - t_L) + d/dx (local sum of lags m >= 0 + u_H) of the forward
// densities at x_j and Dadj the same derivative of the adjoint field (sources
// q and e, local sum signed by sign(x_j - x_source)).  The forward densities
// of each segment of `checkpoint_every` levels are recomputed from the
// checkpoint that starts it.

void grad_setup(wfp_plan* P) {
  if (P->grad_ready) return;
  const int64_t M = P->M, R = P->R, C = P->ckpt_every;
  hipStream_t s = P->stream;
  if (C > 0) {
    // the forward replay's state and the segment's densities after the
    // NQ - 1 levels before it (row NQ - 1 + L - a); recorded levels need neither
    P->rhist = P->alloc<double>((size_t)P->NH * M);
    P->rring = P->alloc<double2>((size_t)P->W * P->npos);
    P->ralpha = P->alloc<double2>(P->npos);
    P->rdalpha = P->alloc<double2>(P->npos);
    P->segsig = P->alloc<double>((size_t)(C + P->NQ - 1) * M);
  }
  P->ahist = P->alloc<double>((size_t)P->NH * M);
  P->aring = P->alloc<double2>((size_t)P->W * P->npos);
  P->aalpha = P->alloc<double2>(P->npos);
  P->adalpha = P->alloc<double2>(P->npos);
  P->gb_acc = P->alloc<double>(M);
  P->gx_acc = P->alloc<double>(M);
  P->xloc = P->alloc<double>(M);
  P->xloc2 = P->alloc<double>(M);
  P->xw = P->alloc<double>(M);
  dterm_setup(P);
  P->esort = P->alloc<double>(R);
  // receivers as spreading sources, in ascending x
  std::vector<int> ord(R);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) { return P->xr_h[a] < P->xr_h[c]; });
  std::vector<double> xrs(R);
  for (int64_t i = 0; i < R; ++i) xrs[i] = P->xr_h[ord[i]];
  std::vector<int> cs(P->nf), cc(P->nf);
  std::vector<int64_t> wo(P->nf);
  int64_t wt = 0;
  for (int i = 0; i < P->nf; ++i) {
    const double xc = -kPi + (double)i * P->hf;
    source_range(xrs, xc, P->alpha_es * (1.0 + 1e-12), true, true, cs[i], cc[i]);
    wo[i] = wt;
    wt += cc[i];
  }
  P->rsort = P->alloc<int>(R);
  P->rcs = P->alloc<int>(P->nf);
  P->rcc = P->alloc<int>(P->nf);
  P->rwo = P->alloc<int64_t>(P->nf);
  P->rsw = P->alloc<double>(wt);
  double* xrs_d = P->alloc<double>(R);
  upload(P->rsort, ord, s);
  upload(P->rcs, cs, s);
  upload(P->rcc, cc, s);
  upload(P->rwo, wo, s);
  upload(xrs_d, xrs, s);
  hipLaunchKernelGGL(k_spread_weights, dim3(nblk(P->nf, 256)), dim3(256), 0, s, P->nf, P->hf, 1.0 / P->alpha_es,
                     P->beta_es, xrs_d, (int)R, P->rcs, P->rcc, P->rwo, P->rsw);
  HIPCHK(hipGetLastError());
  // for every scatterer, the receivers within delta: (r, index in r's list)
  std::vector<std::vector<std::pair<int, int>>> lists(M);
  for (int64_t r = 0; r < R; ++r)
    for (int i = 0; i < P->rnbc_h[r]; ++i) lists[(P->rnbs_h[r] + i) % M].push_back({(int)r, i});
  std::vector<int> ptr(M + 1, 0), rr, ri;
  for (int64_t j = 0; j < M; ++j) {
    for (auto& e : lists[j]) {
      rr.push_back(e.first);
      ri.push_back(e.second);
    }
    ptr[j + 1] = (int)rr.size();
  }
  P->adj_ptr = P->alloc<int>(M + 1);
  P->adj_rr = P->alloc<int>(rr.size());
  P->adj_ri = P->alloc<int>(ri.size());
  upload(P->adj_ptr, ptr, s);
  upload(P->adj_rr, rr, s);
  upload(P->adj_ri, ri, s);
  HIPCHK(hipStreamSynchronize(s));
  P->release(xrs_d);
  P->grad_ready = true;
}

// Weights stored per ordered pair: the signed derivative weights in the
// layout of the weights (same source ranges, lags 0 .. NQ - 1).
void gradx_setup_per_pair(wfp_plan* P, const double* halfs) {
  const int64_t M = P->M;
  hipStream_t s = P->stream;
  double* tmp = P->alloc<double>(P->dense_total);
  launch_local_weights(P, (int)M, P->xs, P->nb_start, P->nb_count, P->qoff, halfs, 1, nullptr, nullptr, tmp);
  std::vector<unsigned> ach((size_t)M * P->NQ);
  HIPCHK(hipMemcpyAsync(ach.data(), P->ac, ach.size() * sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int64_t> rb(M);
  std::vector<uint2> acxh((size_t)M * P->NQ);
  int64_t packed = 0;
  for (int64_t j = 0; j < M; ++j) {
    rb[j] = packed;
    unsigned within = 0;
    for (int m = 0; m < P->NQ; ++m) {
      const unsigned v = ach[(size_t)j * P->NQ + m];
      acxh[(size_t)j * P->NQ + m] = make_uint2(v, within);
      within += v >> 16;
    }
    packed += within;
  }
  P->drowbase = P->alloc<int64_t>(M);
  P->acxd = P->alloc<uint2>(acxh.size());
  P->DQa = P->alloc<double>(packed + 2);   // spare elements for paired loads
  upload(P->drowbase, rb, s);
  upload(P->acxd, acxh, s);
  hipLaunchKernelGGL(k_pack_weights, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ, 0,
                     P->nb_count, P->qoff, tmp, P->ac, P->drowbase, P->DQa);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  P->release(tmp);
}

// Weights stored once per unordered pair: each row's signed derivative
// weights against its upper range, per lag the run of sources that carry it
// (from the row itself), packed; the row and column buffers of the two sums.
void gradx_setup_pair_once(wfp_plan* P, const double* halfs) {
  const int64_t M = P->M;
  hipStream_t s = P->stream;
  std::vector<int> up(M), ust(M), ucnt(M);
  HIPCHK(hipMemcpyAsync(up.data(), P->otf_up_end, M * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int64_t> uoff(M);
  int64_t tot_up = 0, np_up = 0;
  for (int64_t j = 0; j < M; ++j) {
    ust[j] = (int)j;
    ucnt[j] = up[j] - (int)j;
    uoff[j] = tot_up;
    tot_up += (int64_t)ucnt[j] * P->NQ;
    np_up += ucnt[j];
  }
  int* ust_d = P->alloc<int>(M);
  int* ucnt_d = P->alloc<int>(M);
  int64_t* uoff_d = P->alloc<int64_t>(M);
  signed char* umlo = P->alloc<signed char>(np_up);
  double* dense = P->alloc<double>(tot_up);
  unsigned* uac = P->alloc<unsigned>((size_t)M * P->NQ);
  upload(ust_d, ust, s);
  upload(ucnt_d, ucnt, s);
  upload(uoff_d, uoff, s);
  launch_local_weights(P, (int)M, P->xs, ust_d, ucnt_d, uoff_d, halfs, 1, P->sym_upb, umlo, dense);
  hipLaunchKernelGGL(k_row_ranges, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ, ucnt_d,
                     P->sym_upb, umlo, uac);
  HIPCHK(hipGetLastError());
  std::vector<unsigned> ach((size_t)M * P->NQ);
  HIPCHK(hipMemcpyAsync(ach.data(), uac, ach.size() * sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  std::vector<int64_t> rb(M);
  std::vector<uint2> acxh((size_t)M * P->NQ);
  int64_t packed = 0;
  for (int64_t j = 0; j < M; ++j) {
    rb[j] = packed;
    unsigned within = 0;
    for (int m = 0; m < P->NQ; ++m) {
      const unsigned v = ach[(size_t)j * P->NQ + m];
      const unsigned c = v >> 16;
      if (c > 0 && (v & 0xffffu) != 0)
        fail(WFP_EINVAL, "pair-once derivative weights: a lag's sources do not start at the row");
      acxh[(size_t)j * P->NQ + m] = make_uint2(c, within);
      within += c;
    }
    packed += within;
  }
  P->symd_rb = P->alloc<int64_t>(M);
  P->symd_acx = P->alloc<uint2>(acxh.size());
  P->symd_q = P->alloc<double>(packed + 2);
  upload(P->symd_rb, rb, s);
  upload(P->symd_acx, acxh, s);
  hipLaunchKernelGGL(k_pack_weights, dim3(nblk(M, kRowThreads / 64)), dim3(kRowThreads), 0, s, (int)M, P->NQ, 0,
                     ucnt_d, uoff_d, dense, uac, P->symd_rb, P->symd_q);
  HIPCHK(hipGetLastError());
  P->symd_row1 = P->alloc<double>(M);
  P->symd_row2 = P->alloc<double>(M);
  P->symd_col1 = P->alloc<double>(np_up);
  P->symd_col2 = P->alloc<double>(np_up);
  P->symd_one = P->alloc<double>(M);
  upload(P->symd_one, std::vector<double>(M, 1.0), s);
  HIPCHK(hipStreamSynchronize(s));
  for (void* q : {(void*)dense, (void*)uac, (void*)umlo, (void*)ust_d, (void*)ucnt_d, (void*)uoff_d}) P->release(q);
}

// Dynamic LDS of the on-the-fly derivative sums: both histories of a chunk
// and the three column sums of its rows.
size_t otf_deriv_lds(const wfp_plan* P) {
  return (size_t)(2 * P->NQ + 3 * kOtfRows) * kOtfDerivChunk * sizeof(double);
}

// Static LDS of the same kernel: the window table, both row histories side
// by side and their slot tables, plus room for the arrays' alignment.
constexpr size_t kOtfDerivStaticLds = (size_t)kPhiPieces * (kPhiDeg + 1) * sizeof(double) +
                                      (size_t)kOtfRows * (kMaxOtfLags + 1) * sizeof(double2) +
                                      2 * (size_t)(kMaxOtfLags + 1) * sizeof(int64_t) + 64;

// Signed derivative weights for the position gradient, (1/2) dQ_m/dd times
// the sign of x_target - x_source: scatterer rows with lags m >= 0 (per
// ordered pair in the layout of the weights, or once per pair), receivers in
// the layout of their weights with the sign of x_source - x_receiver.
void gradx_setup(wfp_plan* P) {
  if (P->gradx_ready) return;
  // on the fly, the derivative sums stage m_max lags of two histories per
  // chunk in LDS (refused before anything is allocated)
  if (!P->sym_stored && P->otf && otf_deriv_lds(P) + kOtfDerivStaticLds > 160 * 1024)
    fail(WFP_EDOMAIN, "on-the-fly position gradient: too many lags for the LDS stage (W + p/2 > 46)");
  const int64_t M = P->M, R = P->R;
  hipStream_t s = P->stream;
  double* hs = P->alloc<double>(std::max(M, R));
  std::vector<double> halfs(std::max(M, R), 0.5);
  upload(hs, halfs, s);
  if (P->sym_stored) {
    gradx_setup_pair_once(P, hs);
  } else if (P->otf) {
    // on the fly: only the row and column buffers of the two sums
    const size_t lds = otf_deriv_lds(P);
    const void* fns[6] = {(const void*)k_local_otf_deriv2<2>, (const void*)k_local_otf_deriv2<4>,
                          (const void*)k_local_otf_deriv2<6>, (const void*)k_local_otf_deriv2<8>,
                          (const void*)k_local_otf_deriv2<10>, (const void*)k_local_otf_deriv2<12>};
    for (const void* f : fns) HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    P->otfd_row1 = P->alloc<double>(M);
    P->otfd_row2 = P->alloc<double>(M);
    P->otfd_part1 = P->alloc<double>(std::max<int64_t>(P->otf_tot_part, 1));
    P->otfd_part2 = P->alloc<double>(std::max<int64_t>(P->otf_tot_part, 1));
    P->otfd_row3 = P->alloc<double>(M);
    P->otfd_part3 = P->alloc<double>(std::max<int64_t>(P->otf_tot_part, 1));
    P->otfd_next = P->alloc<double>(M);
    P->symd_one = P->alloc<double>(M);
    upload(P->symd_one, std::vector<double>(M, 1.0), s);
  } else {
    gradx_setup_per_pair(P, hs);
  }
  std::vector<double> mhalf(R, -0.5);
  double* mh = P->alloc<double>(R);
  upload(mh, mhalf, s);
  int64_t rt = 0;
  for (int64_t r = 0; r < R; ++r) rt += (int64_t)P->rnbc_h[r] * P->NQ;
  P->dQr = P->alloc<double>(rt);
  launch_local_weights(P, (int)R, P->xr, P->rnb_start, P->rnb_count, P->rqoff, mh, 1, nullptr, nullptr, P->dQr);
  if (P->ckpt_every > 0) P->segD = P->alloc<double>((size_t)P->ckpt_every * M);
  HIPCHK(hipStreamSynchronize(s));
  P->release(hs);
  P->release(mh);
  P->gradx_ready = true;
}

// Buffers of the forward derivative term: f' at the springs, d/dx u_H on the
// fine grid and its modes.
void dterm_setup(wfp_plan* P) {
  if (P->fprime) return;
  P->fprime = P->alloc<double>(P->M);
  P->gridd = P->alloc<double>(P->nf);
  P->yd = P->alloc<double2>(P->K + 1);
}

void deriv_field(wfp_plan* P, const StateRef& S);

// The part of D_j^L that needs the forward state right after level L (held by
// S): f'(x_j - t_L) + d/dx u_H at x_j.  The derivative local sum of the
// forward densities is formed in the backward sweep, in the same pass over the
// derivative weights as the adjoint one.
void fwd_dterm(wfp_plan* P, const StateRef& S, int64_t L, double* out) {
  hipStream_t s = P->stream;
  const int M = (int)P->M;
  const Packets pk{P->npk, 1, P->packets};
  int pp = 1;
  while (pp < P->npk) pp *= 2;
  hipLaunchKernelGGL(k_incident, dim3(nblk(M, 256 / pp)), dim3(256), 0, s, M, (double)L * P->dt, P->xs, P->beta,
                     pk, pp, 1, P->fprime);
  deriv_field(P, S);
  hipLaunchKernelGGL(k_fwd_dterm, dim3(nblk(M, 256)), dim3(256), 0, s, M, P->fprime, P->i0s, P->iw, P->gridd,
                     P->nf, P->width, out);
}

// d/dx u_H at the scatterers' grid: modes -i k alpha_k through the type-2
// transform into P->gridd.
void deriv_field(wfp_plan* P, const StateRef& S) {
  hipStream_t s = P->stream;
  const unsigned nb_b = (unsigned)(P->n2 / 2 + 1);
  const size_t lds_b = P->lds_b;
  hipLaunchKernelGGL(k_deriv_y, dim3(nblk(P->K + 1, 256)), dim3(256), 0, s, P->K, P->n1, P->n2, S.alpha, P->dk2,
                     P->yd);
  hipLaunchKernelGGL(k_hist_b, dim3(nb_b), dim3(512), lds_b, s, 2, P->fft_n1, P->n2, P->K, P->W, (int64_t)0,
                     P->npos, P->T1, P->tw, P->tw1, P->dk1, P->dk2, P->pk, P->qk, P->rot, S.ring, S.alpha,
                     S.dalpha, P->yd, P->V, P->fir_groups, P->hist_threads == 1024 ? 1 : 0);
  launch_hist_c(P, s, (double2*)P->gridd);
}

// Both derivative local sums of a gradient level with the weights on the fly:
// forward densities from rows r1 - m of `fwd`, adjoint ones from the adjoint
// ring at level L2 - m, into P->xloc2 and P->xloc; and, in the same pass, the
// explicit local sum of adjoint level L2 + 1 (scaled by beta/2 as the march's
// own) into P->otfd_next.
void launch_otf_deriv2(wfp_plan* P, hipStream_t s, const double* fwd, int64_t r1, int64_t L2) {
  const int nblocks = 8 * (int)nblk(P->otf_nblk, 8);
  const int periodic = P->boundary == WFP_PERIODIC ? 1 : 0;
  const size_t lds = otf_deriv_lds(P);
#define WFP_OTFD(PP)                                                                                           \
  hipLaunchKernelGGL(k_local_otf_deriv2<PP>, dim3(nblocks), dim3(64 * kOtfRows), lds, s, (int)P->M, P->NH,      \
                     P->NQ, P->otf_up_end, P->otf_blk_end, P->otf_part_off, P->otf_nblk, P->xs, fwd, r1,        \
                     (const double*)P->ahist, L2, periodic, P->dt, P->delta, P->W, P->ngl, P->otf_na, P->otf_nw, \
                     P->phitab, P->otfd_row1, P->otfd_row2, P->otfd_row3, P->otfd_part1, P->otfd_part2,      \
                     P->otfd_part3)
  switch (P->p) {
    case 2: WFP_OTFD(2); break;
    case 4: WFP_OTFD(4); break;
    case 6: WFP_OTFD(6); break;
    case 8: WFP_OTFD(8); break;
    case 10: WFP_OTFD(10); break;
    default: WFP_OTFD(12); break;
  }
#undef WFP_OTFD
  hipLaunchKernelGGL(k_local_otf_reduce, dim3(nblk(P->M, 256)), dim3(256), 0, s, (int)P->M, P->otf_nblk, periodic,
                     P->otf_blk_end, P->otf_part_off, P->otfd_row1, P->otfd_part1, P->symd_one, P->xloc2);
  hipLaunchKernelGGL(k_local_otf_reduce, dim3(nblk(P->M, 256)), dim3(256), 0, s, (int)P->M, P->otf_nblk, periodic,
                     P->otf_blk_end, P->otf_part_off, P->otfd_row2, P->otfd_part2, P->symd_one, P->xloc);
  hipLaunchKernelGGL(k_local_otf_reduce, dim3(nblk(P->M, 256)), dim3(256), 0, s, (int)P->M, P->otf_nblk, periodic,
                     P->otf_blk_end, P->otf_part_off, P->otfd_row3, P->otfd_part3, P->half_beta, P->otfd_next);
  HIPCHK(hipGetLastError());
}

void run_adjoint(wfp_plan* P, int64_t N, const double* e, double* grad_beta, double* grad_x) {
  hipStream_t s = P->stream;
  // recorded levels: the blocks written by the forward run; else each segment
  // is replayed from the checkpoint that starts it
  const bool recorded = P->ckpt_every < 0;
  const int64_t M = P->M, R = P->R, C = recorded ? -(int64_t)P->ckpt_every : P->ckpt_every;
  const bool wx = grad_x != nullptr;
  grad_setup(P);
  if (wx) gradx_setup(P);
  const StateRef rep{P->rhist, P->rring, P->ralpha, P->rdalpha};
  const StateRef adj{P->ahist, P->aring, P->aalpha, P->adalpha};
  const ExtraSources none{nullptr, 0, nullptr, nullptr, nullptr, nullptr};
  zero_state_ref(P, adj);
  // weights on the fly: each level's derivative pass also forms the next
  // adjoint level's local sum (none before the first)
  const bool fused = wx && P->otf && !P->sym_stored;
  bool next_ready = false;
  hipLaunchKernelGGL(k_fill, dim3(nblk(M, 256)), dim3(256), 0, s, P->gb_acc, M, 0.0);
  hipLaunchKernelGGL(k_fill, dim3(nblk(M, 256)), dim3(256), 0, s, P->gx_acc, M, 0.0);
  const int64_t nseg = (N + C - 1) / C;
  const int hd = P->NQ - 1;   // levels kept before the segment
  for (int64_t sg = nseg - 1; sg >= 0; --sg) {
    const int64_t a = sg * C, b = std::min(N, a + C);
    double* const segsig = recorded ? P->rec_sig[(size_t)sg] : P->segsig;
    double* const segD = recorded ? P->rec_D[(size_t)sg] : P->segD;
    if (!recorded) {
      if (sg == 0) zero_state_ref(P, rep);
      else copy_state(P, rep, P->ckpts[(size_t)sg - 1], false);
      hipLaunchKernelGGL(k_seg_head, dim3(nblk((int64_t)hd * M, 256)), dim3(256), 0, s, (int)M, P->NH, a, hd,
                         P->rhist, segsig);
      for (int64_t L = a; L < b; ++L) {
        march_level(P, rep, L, false, none, nullptr, nullptr);
        HIPCHK(hipMemcpyAsync(segsig + (hd + L - a) * M, P->rhist + (L % P->NH) * M, M * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
        if (wx) fwd_dterm(P, rep, L, segD + (L - a) * M);
      }
    }
    for (int64_t L = b - 1; L >= a; --L) {
      const int64_t Rv = N - 1 - L;
      hipLaunchKernelGGL(k_adj_drive, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, (int)R, P->NQ, L, N, P->adj_ptr,
                         P->adj_rr, P->adj_ri, P->rqoff, P->rnb_count, P->Qr, wx ? P->dQr : nullptr, e, P->beta,
                         P->ginc, wx ? P->xw : nullptr);
      ExtraSources ex = none;
      if (L + 1 < N) {
        hipLaunchKernelGGL(k_gather, dim3(nblk(R, 256)), dim3(256), 0, s, (int)R, P->rsort, e + (L + 1) * R,
                           P->esort);
        ex = ExtraSources{P->esort, (int)R, P->rcs, P->rcc, P->rwo, P->rsw};
      }
      march_level(P, adj, Rv, true, ex, nullptr, nullptr, false, false, next_ready ? P->otfd_next : nullptr);
      if (wx) {
        deriv_field(P, adj);
        if (P->sym_stored) {
          hipLaunchKernelGGL(P->sym_spl == 2 ? k_local_sym_deriv2<2> : k_local_sym_deriv2<1>,
                             dim3(8 * nblk(nblk(M, 4), 8)), dim3(256), 0, s, (int)M, P->NQ,
                             P->NH, P->otf_up_end, (const double*)segsig, (int64_t)(hd + L - a),
                             (const double*)P->ahist, Rv, P->symd_rb, P->symd_acx, P->symd_q, P->sym_upb,
                             P->symd_row1, P->symd_row2, P->symd_col1, P->symd_col2);
          hipLaunchKernelGGL(k_local_sym_reduce, dim3(nblk(M, 64)), dim3(64 * kReduceWaves), 0, s, (int)M, P->sym_cov, P->sym_upb,
                             P->symd_row1, P->symd_col1, P->symd_one, P->xloc2);
          hipLaunchKernelGGL(k_local_sym_reduce, dim3(nblk(M, 64)), dim3(64 * kReduceWaves), 0, s, (int)M, P->sym_cov, P->sym_upb,
                             P->symd_row2, P->symd_col2, P->symd_one, P->xloc);
        } else if (P->otf) {
          launch_otf_deriv2(P, s, segsig, (int64_t)(hd + L - a), Rv);
          next_ready = fused;
        } else {
          const int nlocblk = 8 * (int)nblk(nblk(M, kRowThreads / 64), 8);
          hipLaunchKernelGGL(k_local_deriv2, dim3(nlocblk), dim3(kRowThreads), 0, s, (int)M, P->NQ, P->NH,
                             P->nb_start, P->drowbase, P->acxd, P->DQa, (const double*)segsig,
                             (int64_t)(hd + L - a), (const double*)P->ahist, Rv, P->xloc2, P->xloc);
        }
      }
      hipLaunchKernelGGL(k_adj_grad, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, P->ahist + (Rv % P->NH) * M,
                         segsig + (hd + L - a) * M, P->beta, wx ? segD + (L - a) * M : nullptr, P->xloc2,
                         P->xloc, P->xw, P->i0s, P->iw, P->gridd, P->nf, P->width, P->gb_acc,
                         wx ? P->gx_acc : nullptr);
    }
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_unsort, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, P->perm, P->gb_acc, grad_beta);
  if (wx) hipLaunchKernelGGL(k_unsort, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, P->perm, P->gx_acc, grad_x);
  HIPCHK(hipGetLastError());
}


}  // namespace

namespace wfpi {
wfp_status guard(const std::function<void()>& f) {
  try {
    f();
    return WFP_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return WFP_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return WFP_EHIP;
  }
}
}  // namespace wfpi

extern "C" {

wfp_status wfp_plan_create(const wfp_problem* prob, const wfp_params* par, void* stream, wfp_plan** out) {
  if (!out) {
    g_last_error = "out is NULL";
    return WFP_EINVAL;
  }
  *out = nullptr;
  wfp_plan* P = nullptr;
  wfp_status st = guard([&] {
    validate(prob, par);
    P = new wfp_plan();
    HIPCHK(hipGetDevice(&P->device));
    P->stream = (hipStream_t)stream;
    build(P, prob, par);
  });
  if (st != WFP_OK) {
    delete P;
    return st;
  }
  *out = P;
  return WFP_OK;
}

void wfp_plan_destroy(wfp_plan* plan) {
  if (!plan) return;
  (void)hipStreamSynchronize(plan->stream);
  delete plan;
}

wfp_status wfp_plan_info(const wfp_plan* P, wfp_info* info) {
  if (!P || !info) {
    g_last_error = "NULL argument";
    return WFP_EINVAL;
  }
  std::memset(info, 0, sizeof(*info));
  info->M = P->M;
  info->R = P->R;
  info->K = P->K;
  info->n_fine = P->nf;
  info->n_pairs = P->n_pairs;
  info->n_pairs_recv = P->n_pairs_recv;
  info->level = P->level;
  info->W = P->W;
  info->p = P->p;
  info->m_max = P->NH;
  info->n_gl_local = P->ngl;
  info->rbc_period = P->rbc_period;
  info->nufft_width = P->width;
  info->solve_iters = P->iters;
  info->boundary = P->boundary;
  info->dt = P->dt;
  info->delta = P->delta;
  info->b = P->b;
  info->solve_contraction = P->contraction;
  info->device_bytes = P->dev_bytes;
  info->n_weights_nonzero = P->n_weights_nonzero;
  info->n_weights_stored = P->n_weights_stored;
  info->solve_mode = P->solve_global ? 1 : 0;
  info->overlap_cus = P->overlap_cus;
  info->local_mode = P->sym_stored ? 3 : (P->otf ? 2 : 1);
  info->n_weights_lag1 = P->n_weights_lag1;
  info->n_solve_tiles = P->solve_global ? 0 : P->ntile;
  info->n_direct_tiles = P->solve_global ? 0 : P->n_direct_tiles;
  info->sweep_wave = (P->solve_global && P->g_wave) ? 1 : 0;
  return WFP_OK;
}

wfp_status wfp_set_profiling(wfp_plan* P, int32_t enable) {
  if (!P) {
    g_last_error = "NULL plan";
    return WFP_EINVAL;
  }
  return guard([&] {
    flush_profile(P);
    P->profiling = enable != 0;
    if (P->profiling)
      for (int i = 0; i < WFP_N_STAGES; ++i) {
        P->prof_ms[i] = 0;
        P->prof_n[i] = 0;
      }
  });
}

wfp_status wfp_get_profile(wfp_plan* P, double* ms, int64_t* launches) {
  if (!P) {
    g_last_error = "NULL plan";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipStreamSynchronize(P->stream));
    flush_profile(P);
    for (int i = 0; i < WFP_N_STAGES; ++i) {
      if (ms) ms[i] = P->prof_ms[i];
      if (launches) launches[i] = P->prof_n[i];
    }
  });
}

namespace {
// The newest density level and alpha, alpha' checked for NaN or Inf; waits
// for the plan's stream.
void check_finite(wfp_plan* P) {
  hipStream_t s = P->stream;
  if (!P->flag_ext && !P->finite_flag) P->finite_flag = P->alloc<int>(1);
  int* flag = P->flag_ext ? P->flag_ext : P->finite_flag;
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, s, flag, 1, 0);
  const double* newest = P->hist + (int64_t)((P->level - 1) % P->NH) * P->M;
  const int64_t na = 2 * P->npos;
  hipLaunchKernelGGL(k_check_finite, dim3(std::min<int64_t>(nblk(P->M, 256), 1024)), dim3(256), 0, s, newest,
                     P->M, (const double*)P->alpha, na, flag);
  hipLaunchKernelGGL(k_check_finite, dim3(std::min<int64_t>(nblk(na, 256), 1024)), dim3(256), 0, s,
                     (const double*)P->dalpha, na, nullptr, 0, flag);
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (bad) fail(WFP_ENONFINITE, "non-finite densities or mode state after level " + std::to_string(P->level));
}
}  // namespace

wfp_status wfp_run(wfp_plan* P, int64_t n_steps, double* sigma_out, int64_t save_every, double* u_recv_out) {
  if (!P || n_steps < 0) {
    g_last_error = "bad plan or step count";
    return WFP_EINVAL;
  }
  if (sigma_out && save_every < 1) {
    g_last_error = "save_every must be >= 1";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    run_levels(P, n_steps, sigma_out, sigma_out ? save_every : 1, u_recv_out);
    if (P->check_finite && n_steps > 0) check_finite(P);
  });
}

wfp_status wfp_run_noalloc(wfp_plan* P, int64_t n_steps, double* sigma_out, int64_t save_every,
                           double* u_recv_out) {
  if (!P || n_steps < 0) {
    g_last_error = "bad plan or step count";
    return WFP_EINVAL;
  }
  if (sigma_out && save_every < 1) {
    g_last_error = "save_every must be >= 1";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    if (P->ckpt_every != 0)
      fail(WFP_EINVAL, "wfp_run_noalloc: plans that store checkpoints or record levels allocate them; use wfp_run");
    if (P->profiling) fail(WFP_EINVAL, "wfp_run_noalloc: stage timing creates events; use wfp_run");
    if ((size_t)P->M > kScratchDoubles - kScratchHead)
      fail(WFP_EINVAL, "wfp_run_noalloc: M above " + std::to_string(kScratchDoubles - kScratchHead) +
                           " springs (the scratch holds one level of driving data)");
    double* sc = device_scratch(P->device);
    struct Restore {
      wfp_plan* P;
      ~Restore() {
        P->g_ext = nullptr;
        P->g_ext_chunk = 0;
        P->flag_ext = nullptr;
        P->g_lvl0 = -1;
      }
    } restore{P};
    // another call may have left other data there: the block is recomputed
    P->g_ext = sc + kScratchHead;
    P->g_ext_chunk = (int)std::min<int64_t>(256, (int64_t)((kScratchDoubles - kScratchHead) / (size_t)P->M));
    P->flag_ext = (int*)sc;
    P->g_lvl0 = -1;
    run_levels(P, n_steps, sigma_out, sigma_out ? save_every : 1, u_recv_out);
    if (P->check_finite && n_steps > 0) check_finite(P);
  });
}

wfp_status wfp_run_driven(wfp_plan* P, int64_t n_steps, const double* g, double* sigma_out, int64_t save_every,
                          double* u_recv_out) {
  if (!P || n_steps < 0 || (n_steps > 0 && !g)) {
    g_last_error = "bad plan, step count or driving data";
    return WFP_EINVAL;
  }
  if (sigma_out && save_every < 1) {
    g_last_error = "save_every must be >= 1";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    if (n_steps == 0) return;
    const StateRef S = main_state(P);
    const ExtraSources none{nullptr, 0, nullptr, nullptr, nullptr, nullptr};
    const int64_t M = P->M;
    // the gradient pass replays levels with the incident packets' data
    P->ck_from0 = false;
    for (int64_t i = 0; i < n_steps; ++i) {
      const int64_t L = P->level + i;
      hipLaunchKernelGGL(k_drive_gather, dim3(nblk(M, 256)), dim3(256), 0, P->stream, (int)M, P->perm, g + i * M,
                         P->ginc);
      double* save = (sigma_out && i % save_every == 0) ? sigma_out + (i / save_every) * M : nullptr;
      march_level(P, S, L, true, none, save, u_recv_out ? u_recv_out + i * P->R : nullptr);
    }
    HIPCHK(hipGetLastError());
    P->level += n_steps;
    if (P->check_finite) check_finite(P);
  });
}

wfp_status wfp_local_part(wfp_plan* P, double* out) {
  if (!P || !out) {
    g_last_error = "local_part needs a plan and an output array";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    hipStream_t s = P->stream;
    const int64_t M = P->M;
    if (!P->halfs) {
      P->halfs = P->alloc<double>(M);
      hipLaunchKernelGGL(k_fill, dim3(nblk(M, 256)), dim3(256), 0, s, P->halfs, M, 0.5);
    }
    if (P->otf) {
      launch_local_otf(P, s, P->hist, P->level, P->halfs, P->loc);
    } else {
      launch_local_sum(P, s, P->hist, P->level, 1, P->loc);
      hipLaunchKernelGGL(k_unscale, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, P->beta, P->loc);
    }
    hipLaunchKernelGGL(k_unsort, dim3(nblk(M, 256)), dim3(256), 0, s, (int)M, P->perm, P->loc, out);
    HIPCHK(hipGetLastError());
  });
}

wfp_status wfp_adjoint(wfp_plan* P, int64_t n_levels, const double* dJdu, double* grad_beta, double* grad_x) {
  if (!P || !dJdu || !grad_beta || n_levels < 1) {
    g_last_error = "adjoint needs a plan, n_levels >= 1, dJ/du and grad_beta";
    return WFP_EINVAL;
  }
  if (P->boundary != WFP_PERIODIC) {
    g_last_error = "the gradient pass covers the periodic box only";
    return WFP_EDOMAIN;
  }
  if (P->R < 1) {
    g_last_error = "the gradient pass needs receivers (R >= 1)";
    return WFP_EINVAL;
  }
  if (P->ckpt_every == 0 || !P->ck_from0 || P->level < n_levels) {
    g_last_error = "run the n_levels levels from level 0 with checkpoint_every != 0 first";
    return WFP_ESTATE;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    run_adjoint(P, n_levels, dJdu, grad_beta, grad_x);
  });
}

wfp_status wfp_get_state(wfp_plan* P, int64_t* level, double* hist, double* ring, double* alpha,
                         double* dalpha) {
  if (!P) {
    g_last_error = "NULL plan";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    hipStream_t s = P->stream;
    if (level) *level = P->level;
    if (hist) {
      const int64_t n = (int64_t)P->NH * P->M;
      hipLaunchKernelGGL(k_hist_io, dim3(nblk(n, 256)), dim3(256), 0, s, (int)P->M, P->NH, P->level, 1,
                         P->hist, hist, P->perm);
    }
    if (ring) {
      const int64_t n = (int64_t)P->W * (P->K + 1);
      hipLaunchKernelGGL(k_ring_io, dim3(nblk(n, 256)), dim3(256), 0, s, P->K, P->W, P->level, P->n1, P->n2,
                         P->npos, 1, P->ring, (double2*)ring);
    }
    if (alpha)
      hipLaunchKernelGGL(k_modes_io, dim3(nblk(P->K + 1, 256)), dim3(256), 0, s, P->K, P->n1, P->n2, 1, P->alpha,
                         (double2*)alpha);
    if (dalpha)
      hipLaunchKernelGGL(k_modes_io, dim3(nblk(P->K + 1, 256)), dim3(256), 0, s, P->K, P->n1, P->n2, 1,
                         P->dalpha, (double2*)dalpha);
    HIPCHK(hipGetLastError());
  });
}

wfp_status wfp_set_state(wfp_plan* P, int64_t level, const double* hist, const double* ring,
                         const double* alpha, const double* dalpha) {
  if (!P || !hist || !ring || !alpha || !dalpha || level < 0) {
    g_last_error = "set_state needs a plan, level >= 0 and all four arrays";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    hipStream_t s = P->stream;
    const int64_t nh = (int64_t)P->NH * P->M;
    hipLaunchKernelGGL(k_hist_io, dim3(nblk(nh, 256)), dim3(256), 0, s, (int)P->M, P->NH, level, 0, P->hist,
                       const_cast<double*>(hist), P->perm);
    const int64_t nr = (int64_t)P->W * (P->K + 1);
    hipLaunchKernelGGL(k_ring_io, dim3(nblk(nr, 256)), dim3(256), 0, s, P->K, P->W, level, P->n1, P->n2, P->npos,
                       0, P->ring, (double2*)const_cast<double*>(ring));
    hipLaunchKernelGGL(k_modes_io, dim3(nblk(P->K + 1, 256)), dim3(256), 0, s, P->K, P->n1, P->n2, 0, P->alpha,
                       (double2*)const_cast<double*>(alpha));
    hipLaunchKernelGGL(k_modes_io, dim3(nblk(P->K + 1, 256)), dim3(256), 0, s, P->K, P->n1, P->n2, 0, P->dalpha,
                       (double2*)const_cast<double*>(dalpha));
    HIPCHK(hipGetLastError());
    P->level = level;
    P->ck_from0 = false;   // the checkpoints no longer describe this history
  });
}

wfp_status wfp_reset(wfp_plan* P) {
  if (!P) {
    g_last_error = "NULL plan";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    zero_state(P);
  });
}

wfp_status wfp_plan_autotune(wfp_plan* P, int32_t trial_levels, int32_t* overlap_cus) {
  if (!P || trial_levels < 1) {
    g_last_error = "autotune needs a plan and trial_levels >= 1";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(P->device));
    if (P->level != 0) fail(WFP_ESTATE, "autotune runs from level 0 (call wfp_reset first)");
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, P->device));
    const int ncu = prop.multiProcessorCount;
    int nx = 1;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, P->device) != hipSuccess || nx < 1) nx = 1;
    // one stream, or the chain and solve on 1..4 XCDs' worth of compute units
    std::vector<int> cand{-1};
    if (P->ckpt_every == 0)
      for (int q = 1; q <= 4 && q < nx; ++q) cand.push_back(q * (ncu / nx));
    hipStream_t s = P->stream;
    hipEvent_t a = nullptr, c = nullptr;
    const bool prof = P->profiling;
    const int before = P->overlap_cus;
    // on an error the plan keeps its schedule and profiling state
    struct Restore {
      wfp_plan* P;
      bool prof;
      int cus;
      hipEvent_t* ev[2];
      bool done = false;
      ~Restore() {
        for (hipEvent_t* e : ev)
          if (*e) (void)hipEventDestroy(*e);
        if (!done) {
          P->profiling = prof;
          try {
            set_overlap(P, cus);
          } catch (...) {
          }
        }
      }
    } restore{P, prof, before, {&a, &c}};
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&c));
    P->profiling = false;
    float best = 1e30f;
    int pick = -1;
    for (int cus : cand) {
      set_overlap(P, cus);
      run_levels(P, 2, nullptr, 1, nullptr);          // warm-up levels
      HIPCHK(hipEventRecord(a, s));
      run_levels(P, trial_levels, nullptr, 1, nullptr);
      HIPCHK(hipEventRecord(c, s));
      HIPCHK(hipEventSynchronize(c));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, a, c));
      if (ms < best) {
        best = ms;
        pick = cus;
      }
      zero_state(P);
    }
    P->profiling = prof;
    set_overlap(P, pick);
    restore.done = true;
    zero_state(P);
    HIPCHK(hipStreamSynchronize(s));
    if (overlap_cus) *overlap_cus = P->overlap_cus;
  });
}

const char* wfp_status_string(wfp_status s) {
  switch (s) {
    case WFP_OK: return "ok";
    case WFP_EINVAL: return "invalid argument";
    case WFP_EDOMAIN: return "outside the supported domain";
    case WFP_ENOMEM: return "out of memory";
    case WFP_EHIP: return "HIP runtime error";
    case WFP_ESTATE: return "invalid state";
    case WFP_ENONFINITE: return "non-finite values in the march";
    default: return "unknown status";
  }
}

const char* wfp_last_error(void) { return g_last_error.c_str(); }

int32_t wfp_abi_version(void) { return WFP_ABI_VERSION; }

}  // extern "C"
