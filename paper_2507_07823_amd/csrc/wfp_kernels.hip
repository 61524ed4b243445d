// Device kernels of the WFP march for CDNA4 (gfx950), all in FP64.
//
// Data layout (every per-scatterer array is in ascending-x order):
//   hist  [NH][M]       density history ring, slot (L mod NH) holds sigma^L
//   ring  [W][K+1]      spectra ring, slot (n mod W) holds S^n
//   Q     per target row j with n_j sources starting at sorted index nb_start[j]
//         (circularly): Q[qoff[j] + m*n_j + i], m = 0..NQ-1, i = 0..n_j-1,
//         holding (beta_j/2) Q_m(d) (scatterer rows) or (1/2) Q_m(d) (receivers).
//   grid  fine grid of n_f points x_i = -pi + i h_f (NUFFT, periodic)
#include "wfp_kernels.h"

namespace wfp {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kInvTwoPi = 0.15915494309189533577;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by -i
__device__ __forceinline__ double2 cmul_mi(double2 a) { return make_double2(a.y, -a.x); }
// multiply by +i
__device__ __forceinline__ double2 cmul_pi(double2 a) { return make_double2(-a.y, a.x); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// exponential-of-semicircle spreading kernel psi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| < 1
__device__ __forceinline__ double es_kernel(double z, double beta) {
  const double r = 1.0 - z * z;
  return r > 0.0 ? exp(beta * (sqrt(r) - 1.0)) : 0.0;
}

// Chebyshev series a_0/2 + sum a_k T_k(s) by Clenshaw
__device__ __forceinline__ double cheb(const double* __restrict__ a, int n, double s) {
  double b1 = 0.0, b2 = 0.0;
  for (int k = n - 1; k >= 1; --k) {
    const double b0 = fma(2.0 * s, b1, a[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return fma(s, b1, 0.5 * a[0] - b2);
}

__device__ __forceinline__ int mod_slot(int64_t n, int N) {
  int s = (int)(n % N);
  return s < 0 ? s + N : s;
}

// ---------------------------------------------------------------------------
// LDS Stockham FFT (forward, e^{-}), mixed radix 2/4/5, one workgroup.
// Stage with radix R, Ns = product of earlier radices: butterfly j reads
// buf[j + r n/R], twiddles by e^{-2 pi i r (j mod Ns)/(Ns R)}, writes
// buf[(j/Ns) Ns R + (j mod Ns) + r Ns].  Reads go to registers, a barrier,
// then writes: one LDS buffer of n complex values.
// Twiddle table tw[t] = e^{-2 pi i t / (n tws)}.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void butterfly(double2* v) {
  if constexpr (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const double2 t2 = cadd(v[1], v[3]), t3 = cmul_mi(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else {  // R == 5
    const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
    const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
    const double2 t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const double2 t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const double2 v0 = v[0];
    const double2 a1 = make_double2(v0.x + c1 * t1.x + c2 * t2.x, v0.y + c1 * t1.y + c2 * t2.y);
    const double2 a2 = make_double2(v0.x + c2 * t1.x + c1 * t2.x, v0.y + c2 * t1.y + c1 * t2.y);
    const double2 b1 = make_double2(s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y);
    const double2 b2 = make_double2(s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y);
    v[0] = cadd(v0, cadd(t1, t2));
    v[1] = cadd(a1, cmul_mi(b1));
    v[4] = csub(a1, cmul_mi(b1));
    v[2] = cadd(a2, cmul_mi(b2));
    v[3] = csub(a2, cmul_mi(b2));
  }
}

template <int R>
__device__ __forceinline__ void fft_stage(double2* buf, int n, int Ns, const double2* __restrict__ tw,
                                          int tws) {
  const int nb = n / R;
  const int step = n / (Ns * R);
  double2 v[kFftMaxB][R];
#pragma unroll
  for (int c = 0; c < kFftMaxB; ++c) {
    const int j = threadIdx.x + c * kFftThreads;
    if (j < nb) {
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = buf[j + r * nb];
#pragma unroll
      for (int r = 1; r < R; ++r) v[c][r] = cmul(v[c][r], tw[(int64_t)(r * k * step) * tws]);
      butterfly<R>(v[c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kFftMaxB; ++c) {
    const int j = threadIdx.x + c * kFftThreads;
    if (j < nb) {
      const int k = j % Ns;
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[c][r];
    }
  }
  __syncthreads();
}

__device__ void fft_lds(double2* buf, const FftPlan& fp, const double2* __restrict__ tw, int tws) {
  int Ns = 1;
  for (int s = 0; s < fp.nst; ++s) {
    const int R = fp.radix[s];
    if (R == 4) fft_stage<4>(buf, fp.n, Ns, tw, tws);
    else if (R == 5) fft_stage<5>(buf, fp.n, Ns, tw, tws);
    else fft_stage<2>(buf, fp.n, Ns, tw, tws);
    Ns *= R;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Set-up: one-step kernels p_k, q_k (eq. (pkqkcomp)) at m dt, m = 0..W-1, by an
// N_g-node Gauss-Legendre rule on [0, dt], with dt folded in (eq. (hkcompdisc)),
// and the propagator entries cos(k dt), sin(k dt)/k, -k sin(k dt) (Lemma).
// dphi_tab/ddphi_tab hold phi', phi'' at tau = m dt + mu_q ([W][ng]).
// ---------------------------------------------------------------------------
__global__ void k_pq_tables(int64_t K, int W, int ng, double dt, const double* __restrict__ dphi_tab,
                            const double* __restrict__ ddphi_tab, const double* __restrict__ mu,
                            const double* __restrict__ wmu, double* __restrict__ pk,
                            double* __restrict__ qk, double* __restrict__ rot) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > K) return;
  const double kd = (double)k;
  for (int m = 0; m < W; ++m) {
    double ps = 0.0, qs = 0.0;
    for (int q = 0; q < ng; ++q) {
      const double tau = m * dt + mu[q];
      const double sk_tau = (k == 0) ? tau : sin(kd * tau) / kd;
      const double psi = 2.0 * cos(kd * tau) * dphi_tab[m * ng + q] + sk_tau * ddphi_tab[m * ng + q];
      const double u = dt - mu[q];
      const double sk_u = (k == 0) ? u : sin(kd * u) / kd;
      ps += wmu[q] * sk_u * psi;
      qs += wmu[q] * cos(kd * u) * psi;
    }
    pk[(int64_t)m * (K + 1) + k] = dt * ps;
    qk[(int64_t)m * (K + 1) + k] = dt * qs;
  }
  rot[3 * k + 0] = cos(kd * dt);
  rot[3 * k + 1] = (k == 0) ? dt : sin(kd * dt) / kd;
  rot[3 * k + 2] = -kd * sin(kd * dt);
}

// ---------------------------------------------------------------------------
// Set-up: local weights Q_m(d) of Section 4.1 for every (target, source) pair
// closer than delta.  One block per target row, threads over its sources.
// Node i of the N_L-point rule sits at lag s = W - (W - d/dt)(1 + z_i)/2
// (steps before t_{n+1}); weight ((delta - d)/2) w_i (1 - phi(s dt)); stencil
// the P lags from max(m_min, floor(s) - P/2 + 1); Lagrange weights by
// prefix/suffix products  v_r = lagw_r prod_{q != r} (u - q),  u = s - m0.
// Per-thread accumulators live in LDS: acc[m * blockDim + tid].
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(128)
k_local_weights(int nrows, const double* __restrict__ xt, const double* __restrict__ xs, int M,
                const int* __restrict__ nb_start, const int* __restrict__ nb_count,
                const int64_t* __restrict__ qoff, const double* __restrict__ rowscale, int periodic,
                double dt, double delta, int W, int NQ, int ngl, const double* __restrict__ glz,
                const double* __restrict__ glw, const double* __restrict__ cheb_phi, int ncheb,
                const double* __restrict__ lagw, double* __restrict__ Q) {
  extern __shared__ double acc[];
  const int row = blockIdx.x;
  if (row >= nrows) return;
  const int n = nb_count[row];
  const int st = nb_start[row];
  const double xa = xt[row];
  const double scale = rowscale[row];
  const int64_t base = qoff[row];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i0 = 0; i0 < n; i0 += nt) {
    const int i = i0 + tid;
    for (int m = 0; m < NQ; ++m) acc[m * nt + tid] = 0.0;
    if (i < n) {
      int l = st + i;
      if (l >= M) l -= M;
      double d = fabs(xa - xs[l]);
      if (periodic && d > kPi) d = kTwoPi - d;
      if (d < delta) {
        const double D = d / dt;
        const int mmin = (d < dt) ? 0 : 1;
        const double half = 0.5 * (delta - d);
        for (int q = 0; q < ngl; ++q) {
          const double s = W - (W - D) * (1.0 + glz[q]) / 2.0;
          const double phi = cheb(cheb_phi, ncheb, 2.0 * s / W - 1.0);
          const double om = half * glw[q] * (1.0 - phi);
          int m0 = (int)floor(s) - P / 2 + 1;
          if (m0 < mmin) m0 = mmin;
          const double u = s - m0;
          double pre[P];
          pre[0] = 1.0;
#pragma unroll
          for (int r = 1; r < P; ++r) pre[r] = pre[r - 1] * (u - (r - 1));
          double suf = 1.0;
#pragma unroll
          for (int r = P - 1; r >= 0; --r) {
            const double v = lagw[r] * pre[r] * suf;
            suf *= (u - r);
            acc[(m0 + r) * nt + tid] += om * v;
          }
        }
      }
    }
    if (i < n) {
      for (int m = 0; m < NQ; ++m) Q[base + (int64_t)m * n + i] = scale * acc[m * nt + tid];
    }
  }
}

template __global__ void k_local_weights<2>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, int,
                                            const double*, double*);
template __global__ void k_local_weights<4>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, int,
                                            const double*, double*);
template __global__ void k_local_weights<6>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, int,
                                            const double*, double*);
template __global__ void k_local_weights<8>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, int,
                                            const double*, double*);
template __global__ void k_local_weights<10>(int, const double*, const double*, int, const int*, const int*,
                                             const int64_t*, const double*, int, double, double, int, int,
                                             int, const double*, const double*, const double*, int,
                                             const double*, double*);
template __global__ void k_local_weights<12>(int, const double*, const double*, int, const int*, const int*,
                                             const int64_t*, const double*, int, double, double, int, int,
                                             int, const double*, const double*, const double*, int,
                                             const double*, double*);

// Jacobi contraction bound of the per-step system (I + S): for each row,
// sum_{l != j} |S_jl| / (1 + S_jj) over its nearby sources.
__global__ void k_row_contraction(int M, const int* __restrict__ nb_start, const int* __restrict__ nb_count,
                                  const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                                  const int* __restrict__ near_start, const int* __restrict__ near_count,
                                  double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const int st = nb_start[j];
  int self = j - st;
  if (self < 0) self += M;
  const double diag = 1.0 + Q[qoff[j] + self];
  double off = 0.0;
  const int ns = near_start[j], nc = near_count[j];
  for (int c = 0; c < nc; ++c) {
    int l = ns + c;
    if (l >= M) l -= M;
    if (l == j) continue;
    int i = l - st;
    if (i < 0) i += M;
    off += fabs(Q[qoff[j] + i]);
  }
  out[j] = off / diag;
}

// ---------------------------------------------------------------------------
// Type-1 spreading (gather form, atomics-free): grid_i = sum_j sigma_j psi((x_j - x_i)/alpha)
// over the sorted sources inside the kernel support of cell i.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_spread(int nf, double hf, double inv_alpha, double beta_es, const double* __restrict__ xs,
         const double* __restrict__ sig, int M, const int* __restrict__ cstart,
         const int* __restrict__ ccount, double* __restrict__ grid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const double xc = -kPi + i * hf;
  const int st = cstart[i], cnt = ccount[i];
  double acc = 0.0;
  for (int c = 0; c < cnt; ++c) {
    int j = st + c;
    if (j >= M) j -= M;
    double dx = xs[j] - xc;
    dx -= kTwoPi * rint(dx * kInvTwoPi);
    acc += sig[j] * es_kernel(dx * inv_alpha, beta_es);
  }
  grid[i] = acc;
}

// Real-to-complex transform of the fine grid: z = FFT_{n}(grid[2j] + i grid[2j+1]).
__global__ void __launch_bounds__(1024)
k_fft_r2c(FftPlan fp, const double2* __restrict__ grid, const double2* __restrict__ tw, int tws,
          double2* __restrict__ zout) {
  extern __shared__ double2 buf[];
  for (int j = threadIdx.x; j < fp.n; j += blockDim.x) buf[j] = grid[j];
  __syncthreads();
  fft_lds(buf, fp, tw, tws);
  for (int j = threadIdx.x; j < fp.n; j += blockDim.x) zout[j] = buf[j];
}

// ---------------------------------------------------------------------------
// Mode update for level L (time t_n -> t_{n+1}, n = L-1), one thread per k:
//   X_k (real-FFT unpacking) -> S_k^n = dk1_k conj(X_k)   (eq. (densco) via the type-1 NUFFT)
//   ring[n mod W] = S^n
//   h_k = sum_m pk[m][k] S_k^{n-m},  g_k likewise            (eq. (hkcompdisc))
//   (alpha, alpha') <- propagator + (h, g)                    (Lemma)
//   y_k = dk2_k conj(alpha_k)                                 (type-2 pre-correction)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_modes(int64_t K, int W, int nfh, int64_t L, const double2* __restrict__ z, const double2* __restrict__ tw,
        const double* __restrict__ dk1, const double* __restrict__ dk2, const double* __restrict__ pk,
        const double* __restrict__ qk, const double* __restrict__ rot, double2* __restrict__ ring,
        double2* __restrict__ alpha, double2* __restrict__ dalpha, double2* __restrict__ y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > K) return;
  const double2 zk = z[k];
  const double2 zc = cconj(z[k == 0 ? 0 : nfh - k]);
  const double2 E = cscale(cadd(zk, zc), 0.5);
  const double2 O = cscale(cmul_mi(csub(zk, zc)), 0.5);
  const double2 X = cadd(E, cmul(tw[k], O));
  const double2 S = cscale(cconj(X), dk1[k]);
  const int64_t n = L - 1;
  const int64_t stride = K + 1;
  ring[(int64_t)mod_slot(n, W) * stride + k] = S;
  double2 h = make_double2(0.0, 0.0), g = make_double2(0.0, 0.0);
  for (int m = 0; m < W; ++m) {
    const double2 Sm = (m == 0) ? S : ring[(int64_t)mod_slot(n - m, W) * stride + k];
    const double p = pk[(int64_t)m * stride + k], q = qk[(int64_t)m * stride + k];
    h.x = fma(p, Sm.x, h.x);
    h.y = fma(p, Sm.y, h.y);
    g.x = fma(q, Sm.x, g.x);
    g.y = fma(q, Sm.y, g.y);
  }
  const double c = rot[3 * k], s = rot[3 * k + 1], r = rot[3 * k + 2];
  const double2 a = alpha[k], da = dalpha[k];
  const double2 an = make_double2(c * a.x + s * da.x + h.x, c * a.y + s * da.y + h.y);
  const double2 dan = make_double2(r * a.x + c * da.x + g.x, r * a.y + c * da.y + g.y);
  alpha[k] = an;
  dalpha[k] = dan;
  y[k] = cscale(cconj(an), dk2[k]);
}

// Complex-to-real transform: grid_i = sum_{|k|<=K} y_k e^{+2 pi i i k / N} for
// Hermitian y (given for k = 0..K, zero above), via an n = N/2 complex inverse
// transform of the packed spectrum and conjugation around the forward FFT.
__global__ void __launch_bounds__(1024)
k_fft_c2r(FftPlan fp, int64_t K, const double2* __restrict__ y, const double2* __restrict__ tw, int tws,
          double2* __restrict__ grid_out) {
  extern __shared__ double2 buf[];
  const int n = fp.n;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double2 yk = (k <= K) ? y[k] : make_double2(0.0, 0.0);
    const int km = n - k;
    const double2 ym = (k > 0 && km <= K) ? cconj(y[km]) : make_double2(0.0, 0.0);
    // Z_k = (yk + ym) + i e^{+2 pi i k/N} (yk - ym);  e^{+} = conj(tw[k])
    const double2 zk = cadd(cadd(yk, ym), cmul_pi(cmul(cconj(tw[k]), csub(yk, ym))));
    buf[k] = cconj(zk);
  }
  __syncthreads();
  fft_lds(buf, fp, tw, tws);
  for (int j = threadIdx.x; j < n; j += blockDim.x) grid_out[j] = cconj(buf[j]);
}

// ---------------------------------------------------------------------------
// Right-hand side of the level-L system, one wavefront per scatterer row j:
//   rhs_j = -g_j(t_L) - sum_{m>=1} sum_l (beta_j/2) Q_m(d_jl) sigma_l^{L-m} - beta_j u_H(x_j)
// with u_H(x_j) interpolated from the type-2 grid (lanes over the kernel cells)
// and g_j = beta_j f(x_j - t_L) (eq. (gj); f periodised in the periodic box).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double incident_profile(double s, const Packets& pk) {
  if (pk.periodic) s -= kTwoPi * rint(s * kInvTwoPi);
  double out = 0.0;
  for (int i = 0; i < pk.n; ++i) {
    const double a = pk.p[5 * i], c = pk.p[5 * i + 1], w = pk.p[5 * i + 2];
    const double om = pk.p[5 * i + 3], ph = pk.p[5 * i + 4];
    const double lim = 40.0 * w;   // exp(-y^2/(2w^2)) underflows to 0 beyond
    if (pk.periodic) {
      for (int m = -4; m <= 4; ++m) {
        const double y = (s + kTwoPi * m) - c;
        if (fabs(y) < lim) out += a * exp(-y * y / (2.0 * w * w)) * cos(om * y + ph);
      }
    } else {
      const double y = s - c;
      if (fabs(y) < lim) out += a * exp(-y * y / (2.0 * w * w)) * cos(om * y + ph);
    }
  }
  return out;
}

__device__ __forceinline__ double interp_lane(double x, const double* __restrict__ grid2, int nf, double hf,
                                              double inv_alpha, double beta_es, int width, int lane) {
  // cells i0 .. i0+width-1 with i0 = ceil((x + pi)/hf - width/2)
  double v = 0.0;
  if (lane < width) {
    const int i0 = (int)ceil((x + kPi) / hf - 0.5 * width);
    int i = i0 + lane;
    i %= nf;
    if (i < 0) i += nf;
    double dx = x - (-kPi + i * hf);
    dx -= kTwoPi * rint(dx * kInvTwoPi);
    v = grid2[i] * es_kernel(dx * inv_alpha, beta_es);
  }
  return v;
}

__global__ void __launch_bounds__(256)
k_local_rhs(int M, int NQ, int NH, int64_t L, double t, const double* __restrict__ xs,
            const double* __restrict__ beta, const int* __restrict__ nb_start, const int* __restrict__ nb_count,
            const int64_t* __restrict__ qoff, const double* __restrict__ Q, const double* __restrict__ hist,
            const double* __restrict__ grid2, int nf, double hf, double inv_alpha, double beta_es, int width,
            Packets pk, double* __restrict__ rhs) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= M) return;
  const int n = nb_count[j];
  const int st = nb_start[j];
  const int64_t base = qoff[j];
  double acc = 0.0;
  for (int m = 1; m < NQ; ++m) {
    const double* __restrict__ sl = hist + (int64_t)mod_slot(L - m, NH) * M;
    const double* __restrict__ qm = Q + base + (int64_t)m * n;
    for (int i = lane; i < n; i += 64) {
      int l = st + i;
      if (l >= M) l -= M;
      acc = fma(qm[i], sl[l], acc);
    }
  }
  acc = wave_sum(acc);
  const double x = xs[j];
  const double uh = wave_sum(interp_lane(x, grid2, nf, hf, inv_alpha, beta_es, width, lane));
  if (lane == 0) {
    const double bj = beta[j];
    const double g = bj * incident_profile(x - t, pk);
    rhs[j] = -g - acc - bj * uh;
  }
}

// ---------------------------------------------------------------------------
// Per-step solve (I + S) sigma^L = rhs, S_jl = (beta_j/2) Q_0(d_jl) for d < dt
// (eq. (linearSystem)), by `iters` Jacobi sweeps from zero.  One block per
// tile of T consecutive rows; the block iterates on the tile plus a halo
// holding every point within `iters` couplings of it, so the tile's result is
// identical to `iters` global sweeps.  The result goes to the history slot of
// level L and, when requested, to a row of the caller's output (original order).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_jacobi(int M, int T, int iters, int ext_max, const int* __restrict__ ext_start, const int* __restrict__ ext_len,
         const int* __restrict__ nb_start, const int64_t* __restrict__ qoff, const double* __restrict__ Q,
         const int* __restrict__ near_start, const int* __restrict__ near_count, const double* __restrict__ rhs,
         double* __restrict__ sig_out, double* __restrict__ save_row, const int* __restrict__ perm) {
  extern __shared__ double sm[];
  double* s0 = sm;
  double* s1 = sm + ext_max;
  const int tile = blockIdx.x;
  const int es = ext_start[tile], el = ext_len[tile];
  for (int e = threadIdx.x; e < el; e += blockDim.x) {
    int g = es + e;
    if (g >= M) g -= M;
    int self = g - nb_start[g];
    if (self < 0) self += M;
    s0[e] = rhs[g] / (1.0 + Q[qoff[g] + self]);
  }
  __syncthreads();
  for (int it = 1; it < iters; ++it) {
    for (int e = threadIdx.x; e < el; e += blockDim.x) {
      int g = es + e;
      if (g >= M) g -= M;
      const int st = nb_start[g];
      const int64_t qb = qoff[g];
      int self = g - st;
      if (self < 0) self += M;
      double acc = rhs[g];
      const int ns = near_start[g], nc = near_count[g];
      for (int c = 0; c < nc; ++c) {
        int l = ns + c;
        if (l >= M) l -= M;
        if (l == g) continue;
        int le = l - es;
        if (le < 0) le += M;
        if (le >= el) continue;  // outside the halo: only reaches points that are not kept
        int i = l - st;
        if (i < 0) i += M;
        acc = fma(-Q[qb + i], s0[le], acc);
      }
      s1[e] = acc / (1.0 + Q[qb + self]);
    }
    __syncthreads();
    double* tmp = s0;
    s0 = s1;
    s1 = tmp;
  }
  const int t0 = tile * T;
  for (int c = threadIdx.x; c < T; c += blockDim.x) {
    const int g = t0 + c;
    if (g >= M) break;
    int le = g - es;
    if (le < 0) le += M;
    const double v = s0[le];
    sig_out[g] = v;
    if (save_row) save_row[perm[g]] = v;
  }
}

// Field at the receivers, one wavefront per receiver:
//   u(x_r, t_L) = sum_{m>=0} sum_l (1/2) Q_m(d_rl) sigma_l^{L-m} + u_H(x_r)
__global__ void __launch_bounds__(256)
k_receivers(int R, int M, int NQ, int NH, int64_t L, const double* __restrict__ xr,
            const int* __restrict__ nb_start, const int* __restrict__ nb_count, const int64_t* __restrict__ qoff,
            const double* __restrict__ Q, const double* __restrict__ hist, const double* __restrict__ grid2,
            int nf, double hf, double inv_alpha, double beta_es, int width, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= R) return;
  const int n = nb_count[r];
  const int st = nb_start[r];
  const int64_t base = qoff[r];
  double acc = 0.0;
  for (int m = 0; m < NQ; ++m) {
    const double* __restrict__ sl = hist + (int64_t)mod_slot(L - m, NH) * M;
    const double* __restrict__ qm = Q + base + (int64_t)m * n;
    for (int i = lane; i < n; i += 64) {
      int l = st + i;
      if (l >= M) l -= M;
      acc = fma(qm[i], sl[l], acc);
    }
  }
  acc = wave_sum(acc);
  const double uh = wave_sum(interp_lane(xr[r], grid2, nf, hf, inv_alpha, beta_es, width, lane));
  if (lane == 0) out[r] = acc + uh;
}

// ---------------------------------------------------------------------------
// Free-space RBC projection (Section 4.4).  Block 0 handles alpha -> u,
// block 1 alpha' -> v: values on x_i = -pi + i h, i = 0..2K-1 (h = pi/K), from
// the modes |k| < K (k = K dropped): grid = c2r of y_k = (-1)^k conj(a_k).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_rbc_to_grid(FftPlan fp, int64_t K, const double2* __restrict__ alpha, const double2* __restrict__ dalpha,
              const double2* __restrict__ tw, double2* __restrict__ gu, double2* __restrict__ gv) {
  extern __shared__ double2 buf[];
  const double2* __restrict__ a = (blockIdx.x == 0) ? alpha : dalpha;
  double2* __restrict__ out = (blockIdx.x == 0) ? gu : gv;
  const int n = fp.n;  // == K
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double sk = (k & 1) ? -1.0 : 1.0;
    const double2 yk = cscale(cconj(a[k]), sk);
    const int km = n - k;   // 1..K-1 for k >= 1
    double2 ym = make_double2(0.0, 0.0);
    if (k > 0) {
      const double sm = (km & 1) ? -1.0 : 1.0;
      ym = cconj(cscale(cconj(a[km]), sm));
    }
    const double2 zk = cadd(cadd(yk, ym), cmul_pi(cmul(cconj(tw[k]), csub(yk, ym))));
    buf[k] = cconj(zk);
  }
  __syncthreads();
  fft_lds(buf, fp, tw, 2);
  for (int j = threadIdx.x; j < n; j += blockDim.x) out[j] = cconj(buf[j]);
}

// Roll-off on |i - K| >= K - 2W with the spatial window (delta_s = W h):
//   u~ = phi_s(a) u,  v~ = phi_s'(a) u + phi_s(a) v,  a = (K - |i - K| - W) h,
// then back to modes alpha_k = (1/2K) (-1)^k conj(X_k), k < K, alpha_K = 0.
// Block 0 writes alpha and the type-2 input y, block 1 writes alpha'.
__global__ void __launch_bounds__(1024)
k_rbc_to_modes(FftPlan fp, int64_t K, int W, double h, double delta_s, const double* __restrict__ cheb_phi,
               const double* __restrict__ cheb_g, int ncheb, const double* __restrict__ gu,
               const double* __restrict__ gv, const double2* __restrict__ tw, const double* __restrict__ dk2,
               double2* __restrict__ alpha, double2* __restrict__ dalpha, double2* __restrict__ y) {
  extern __shared__ double2 buf[];
  const int n = fp.n;       // == K complex, 2K real points
  const bool is_v = blockIdx.x == 1;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double val[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int ip = 2 * j + e;          // grid index 0..2K-1
      int i = ip - (int)K;               // -K..K-1
      const int ai = i < 0 ? -i : i;
      double u = gu[ip];
      double v = is_v ? gv[ip] : 0.0;
      if (ai >= (int)K - 2 * W) {
        const double arg = (double)((int)K - ai - W) * h;
        double rho, drho;
        if (arg <= 0.0) rho = 0.0;
        else if (arg >= delta_s) rho = 1.0;
        else rho = cheb(cheb_phi, ncheb, 2.0 * arg / delta_s - 1.0);
        if (arg >= 0.0 && arg <= delta_s) drho = (2.0 / delta_s) * cheb(cheb_g, ncheb, 2.0 * arg / delta_s - 1.0);
        else drho = 0.0;
        if (is_v) v = drho * u + rho * v;
        else u = rho * u;
      }
      val[e] = is_v ? v : u;
    }
    buf[j] = make_double2(val[0], val[1]);
  }
  __syncthreads();
  fft_lds(buf, fp, tw, 2);
  // unpack the real transform of length 2K and return to modes
  const double inv = 1.0 / (2.0 * (double)K);
  double2* __restrict__ out = is_v ? dalpha : alpha;
  for (int k = threadIdx.x; k <= n; k += blockDim.x) {
    double2 a = make_double2(0.0, 0.0);
    if (k < n) {
      const double2 zk = buf[k];
      const double2 zc = cconj(buf[k == 0 ? 0 : n - k]);
      const double2 E = cscale(cadd(zk, zc), 0.5);
      const double2 O = cscale(cmul_mi(csub(zk, zc)), 0.5);
      const double2 X = cadd(E, cmul(tw[k], O));
      const double sk = (k & 1) ? -1.0 : 1.0;
      a = cscale(cconj(X), sk * inv);
    }
    out[k] = a;
    if (!is_v) y[k] = cscale(cconj(a), dk2[k]);
  }
}

// ---------------------------------------------------------------------------
// State movement between the internal rings (sorted order) and user arrays.
// ---------------------------------------------------------------------------
__global__ void k_hist_io(int M, int NH, int64_t L, int to_user, double* __restrict__ hist,
                          double* __restrict__ user, const int* __restrict__ perm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)NH * M) return;
  const int m = (int)(t / M), j = (int)(t % M);
  const int slot = mod_slot(L - 1 - m, NH);
  double* h = hist + (int64_t)slot * M + j;
  double* u = user + (int64_t)m * M + perm[j];
  if (to_user) *u = *h;
  else *h = *u;
}

__global__ void k_ring_io(int64_t K, int W, int64_t L, int to_user, double2* __restrict__ ring,
                          double2* __restrict__ user) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)W * (K + 1)) return;
  const int m = (int)(t / (K + 1));
  const int64_t k = t % (K + 1);
  const int slot = mod_slot(L - 2 - m, W);
  double2* r = ring + (int64_t)slot * (K + 1) + k;
  double2* u = user + (int64_t)m * (K + 1) + k;
  if (to_user) *u = *r;
  else *r = *u;
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace wfp
