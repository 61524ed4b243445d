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

// Storage position of Fourier mode q in every per-mode array (tables, spectra
// ring, alpha, alpha'): the order in which the history kernel's blocks visit
// the modes.  q = k2 + n2 k1 lives in block b = min(k2, n2 - k2) (column pair
// {k2, n2 - k2}), column c = (k2 > n2/2), at b * 2 n1 + c * n1 + k1.
__device__ __forceinline__ int64_t mode_pos(int64_t q, int n1, int n2) {
  const int k2 = (int)(q % n2), k1 = (int)(q / n2);
  const int b = (k2 == 0) ? 0 : min(k2, n2 - k2);
  const int c = (k2 == b) ? 0 : 1;
  return (int64_t)b * 2 * n1 + c * n1 + k1;
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

// Batched variant: nb independent FFTs of length fp.n at buf + b * fp.n, all
// threads of the block taking part (at most kFftMaxB butterflies per thread per
// stage; checked on the host).
template <int R>
__device__ __forceinline__ void fft_stage_batch(double2* buf, int n, int nb, int Ns, const double2* __restrict__ tw,
                                                int tws) {
  const int per = n / R;
  const int tot = per * nb;
  const int step = n / (Ns * R);
  double2 v[kFftMaxB][R];
#pragma unroll
  for (int c = 0; c < kFftMaxB; ++c) {
    const int idx = threadIdx.x + c * blockDim.x;
    if (idx < tot) {
      const int b = idx / per, j = idx - b * per;
      const double2* base = buf + b * n;
      const int k = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[c][r] = base[j + r * per];
#pragma unroll
      for (int r = 1; r < R; ++r) v[c][r] = cmul(v[c][r], tw[(int64_t)(r * k * step) * tws]);
      butterfly<R>(v[c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kFftMaxB; ++c) {
    const int idx = threadIdx.x + c * blockDim.x;
    if (idx < tot) {
      const int b = idx / per, j = idx - b * per;
      double2* base = buf + b * n;
      const int k = j % Ns;
      const int o = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) base[o + r * Ns] = v[c][r];
    }
  }
  __syncthreads();
}

__device__ void fft_batch(double2* buf, int nb, const FftPlan& fp, const double2* __restrict__ tw, int tws) {
  int Ns = 1;
  for (int s = 0; s < fp.nst; ++s) {
    const int R = fp.radix[s];
    if (R == 4) fft_stage_batch<4>(buf, fp.n, nb, Ns, tw, tws);
    else if (R == 5) fft_stage_batch<5>(buf, fp.n, nb, Ns, tw, tws);
    else fft_stage_batch<2>(buf, fp.n, nb, Ns, tw, tws);
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
                            const double* __restrict__ wmu, int n1, int n2, int64_t npos,
                            double* __restrict__ pk, double* __restrict__ qk, double* __restrict__ rot) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > K) return;
  const int64_t pos = mode_pos(k, n1, n2);
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
    pk[(int64_t)m * npos + pos] = dt * ps;
    qk[(int64_t)m * npos + pos] = dt * qs;
  }
  rot[3 * pos + 0] = cos(kd * dt);
  rot[3 * pos + 1] = (k == 0) ? dt : sin(kd * dt) / kd;
  rot[3 * pos + 2] = -kd * sin(kd * dt);
}

// ---------------------------------------------------------------------------
// Set-up: local weights Q_m(d) of Section 4.1 for every (target, source) pair
// closer than delta.  One block per target row, threads over its sources.
// Node i of the N_L-point rule sits at lag s = W - (W - d/dt)(1 + z_i)/2
// (steps before t_{n+1}); weight ((delta - d)/2) w_i (1 - phi(s dt)); stencil
// the P lags from max(m_min, floor(s) - P/2 + 1); Lagrange weights by
// prefix/suffix products  v_r = lagw_r prod_{q != r} (u - q),  u = s - m0.
// Per-thread accumulators live in LDS: acc[m * blockDim + tid]; lags
// 0..nq_out-1 are written.  With deriv != 0 the kernel writes dQ_m/dd times sign(wrap(x_target - x_source))
// instead (for gradients with respect to positions): with ds/dd = (1 + z_i)/(2 dt),
//   d/dd [node weight] = -(1/2) w_i (1 - phi(s dt)) - ((delta - d)/2) w_i phi'(s dt) dt ds/dd,
// and the Lagrange weights differentiated by the product rule (the stencil is
// piecewise constant in d).
// ---------------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(128)
k_local_weights(int nrows, const double* __restrict__ xt, const double* __restrict__ xs, int M,
                const int* __restrict__ nb_start, const int* __restrict__ nb_count,
                const int64_t* __restrict__ qoff, const double* __restrict__ rowscale, int periodic,
                double dt, double delta, int W, int NQ, int ngl, const double* __restrict__ glz,
                const double* __restrict__ glw, const double* __restrict__ cheb_phi,
                const double* __restrict__ cheb_g, int ncheb, int deriv,
                const double* __restrict__ lagw, const int64_t* __restrict__ pbase,
                signed char* __restrict__ mlo, int nq_out, double* __restrict__ Q) {
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
    int lowest = NQ;
    double sgn = 1.0;
    if (i < n) {
      int l = st + i;
      if (l >= M) l -= M;
      double d = fabs(xa - xs[l]);
      if (periodic && d > kPi) d = kTwoPi - d;
      if (deriv) {
        double y = xa - xs[l];
        if (periodic) y -= kTwoPi * rint(y * kInvTwoPi);
        sgn = (y > 0.0) ? 1.0 : ((y < 0.0) ? -1.0 : 0.0);
      }
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
          if (m0 > W - P / 2) m0 = W - P / 2;   // s == W (d within an ulp of delta)
          if (m0 < lowest) lowest = m0;
          const double u = s - m0;
          double pre[P], dpre[P];
          pre[0] = 1.0;
          dpre[0] = 0.0;
#pragma unroll
          for (int r = 1; r < P; ++r) {
            dpre[r] = dpre[r - 1] * (u - (r - 1)) + pre[r - 1];
            pre[r] = pre[r - 1] * (u - (r - 1));
          }
          if (!deriv) {
            double suf = 1.0;
#pragma unroll
            for (int r = P - 1; r >= 0; --r) {
              const double v = lagw[r] * pre[r] * suf;
              suf *= (u - r);
              acc[(m0 + r) * nt + tid] += om * v;
            }
          } else {
            const double ds = (1.0 + glz[q]) / (2.0 * dt);
            const double dphi = (2.0 / delta) * cheb(cheb_g, ncheb, 2.0 * s / W - 1.0);
            const double dom = -0.5 * glw[q] * (1.0 - phi) - half * glw[q] * dphi * dt * ds;
            double suf = 1.0, dsuf = 0.0;
#pragma unroll
            for (int r = P - 1; r >= 0; --r) {
              const double v = lagw[r] * pre[r] * suf;
              const double dv = lagw[r] * (dpre[r] * suf + pre[r] * dsuf);
              dsuf = dsuf * (u - r) + suf;
              suf *= (u - r);
              acc[(m0 + r) * nt + tid] += dom * v + om * dv * ds;
            }
          }
        }
      }
    }
    if (i < n) {
      const double sc = deriv ? scale * sgn : scale;
      for (int m = 0; m < nq_out; ++m) Q[base + (int64_t)m * n + i] = sc * acc[m * nt + tid];
      if (mlo) mlo[pbase[row] + i] = (signed char)lowest;
    }
  }
}

template __global__ void k_local_weights<2>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, const double*, int, int,
                                            const double*, const int64_t*, signed char*, int, double*);
template __global__ void k_local_weights<4>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, const double*, int, int,
                                            const double*, const int64_t*, signed char*, int, double*);
template __global__ void k_local_weights<6>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, const double*, int, int,
                                            const double*, const int64_t*, signed char*, int, double*);
template __global__ void k_local_weights<8>(int, const double*, const double*, int, const int*, const int*,
                                            const int64_t*, const double*, int, double, double, int, int,
                                            int, const double*, const double*, const double*, const double*, int, int,
                                            const double*, const int64_t*, signed char*, int, double*);
template __global__ void k_local_weights<10>(int, const double*, const double*, int, const int*, const int*,
                                             const int64_t*, const double*, int, double, double, int, int,
                                             int, const double*, const double*, const double*, const double*, int, int,
                                             const double*, const int64_t*, signed char*, int, double*);
template __global__ void k_local_weights<12>(int, const double*, const double*, int, const int*, const int*,
                                             const int64_t*, const double*, int, double, double, int, int,
                                             int, const double*, const double*, const double*, const double*, int, int,
                                             const double*, const int64_t*, signed char*, int, double*);

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

// For each row and lag m, the index range [a, a + c) of sources whose lowest
// nonzero lag is <= m (one wavefront per row).  A source at distance d has
// nonzero weights exactly for lags mlo(d)..NQ-1 and mlo grows with d, so the
// range is the contiguous block of neighbours closest to the target.
// Packed as a | (c << 16).
__global__ void k_row_ranges(int M, int NQ, const int* __restrict__ nb_count, const int64_t* __restrict__ pbase,
                             const signed char* __restrict__ mlo, unsigned* __restrict__ ac) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= M) return;
  const int n = nb_count[j];
  const signed char* __restrict__ ml = mlo + pbase[j];
  for (int m = 0; m < NQ; ++m) {
    int lo = 0x7fffffff, hi = -1;
    for (int i = lane; i < n; i += 64)
      if (ml[i] <= m) {
        lo = min(lo, i);
        hi = max(hi, i);
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    if (lane == 0) ac[(int64_t)j * NQ + m] = (hi < 0) ? 0u : ((unsigned)lo | ((unsigned)(hi - lo + 1) << 16));
  }
}

// Copy the weights of lags m >= m0 inside each row's ranges to the packed layout
// Qc[rowbase[j] + sum_{m0 <= m' < m} c_{jm'} + (i - a_jm)].
__global__ void k_pack_weights(int M, int NQ, int m0, const int* __restrict__ nb_count,
                               const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                               const unsigned* __restrict__ ac, const int64_t* __restrict__ rowbase,
                               double* __restrict__ Qc) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= M) return;
  const int n = nb_count[j];
  int64_t off = rowbase[j];
  for (int m = m0; m < NQ; ++m) {
    const unsigned v = ac[(int64_t)j * NQ + m];
    const int a = v & 0xffff, c = v >> 16;
    for (int i = lane; i < c; i += 64) Qc[off + i] = Q[qoff[j] + (int64_t)m * n + a + i];
    off += c;
  }
}

// Values of the solve's tile matrices: off-diagonal couplings and the inverse
// diagonal, gathered from the lag-0 weights.
__global__ void k_gather_solve(int64_t ne, const int64_t* __restrict__ eq, const double* __restrict__ Q,
                               double* __restrict__ ev, int64_t nr, const int64_t* __restrict__ rq,
                               double* __restrict__ rdinv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < ne) ev[t] = Q[eq[t]];
  if (t < nr) rdinv[t] = 1.0 / (1.0 + Q[rq[t]]);
}

// Spreading weights psi((x_j - x_i)/alpha) of every (cell, source) pair in the
// cell's source range, at w[woff_i + c] (the points never move).
__global__ void k_spread_weights(int nf, double hf, double inv_alpha, double beta_es, const double* __restrict__ xs,
                                 int M, const int* __restrict__ cstart, const int* __restrict__ ccount,
                                 const int64_t* __restrict__ woff, double* __restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf) return;
  const double xc = -kPi + i * hf;
  const int st = cstart[i], cnt = ccount[i];
  for (int c = 0; c < cnt; ++c) {
    int j = st + c;
    if (j >= M) j -= M;
    double dx = xs[j] - xc;
    dx -= kTwoPi * rint(dx * kInvTwoPi);
    w[woff[i] + c] = es_kernel(dx * inv_alpha, beta_es);
  }
}

// Interpolation stencil of a target x: first cell i0 = ceil((x + pi)/h_f - width/2)
// and the weights psi((x - x_i)/alpha) of cells i0 .. i0 + width - 1 (mod n_f).
__global__ void k_interp_weights(int n, int nf, double hf, double inv_alpha, double beta_es, int width,
                                 const double* __restrict__ x, int* __restrict__ i0s, double* __restrict__ w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double xj = x[j];
  const int i0 = (int)ceil((xj + kPi) / hf - 0.5 * width);
  i0s[j] = i0;
  for (int q = 0; q < width; ++q) {
    int i = i0 + q;
    i %= nf;
    if (i < 0) i += nf;
    double dx = xj - (-kPi + i * hf);
    dx -= kTwoPi * rint(dx * kInvTwoPi);
    w[(int64_t)j * width + q] = es_kernel(dx * inv_alpha, beta_es);
  }
}

__device__ __forceinline__ double interp_pre(int j, const int* __restrict__ i0s, const double* __restrict__ w,
                                             const double* __restrict__ grid2, int nf, int width) {
  int i = i0s[j] % nf;
  if (i < 0) i += nf;
  double uh = 0.0;
  for (int q = 0; q < width; ++q) {
    uh = fma(w[(int64_t)j * width + q], grid2[i], uh);
    if (++i == nf) i = 0;
  }
  return uh;
}

// Number of nonzero stored weights of lag m >= 1 (one wavefront per row).
__global__ void k_count_nonzero(int M, int NQ, const int* __restrict__ nb_count, const int64_t* __restrict__ qoff,
                                const double* __restrict__ Q, unsigned long long* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= M) return;
  const int n = nb_count[j];
  unsigned long long c = 0;
  for (int64_t e = (int64_t)n + lane; e < (int64_t)NQ * n; e += 64) c += (Q[qoff[j] + e] != 0.0);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (lane == 0) atomicAdd(out, c);
}

// XCD-aware block order: consecutive hardware block ids go round-robin over
// the 8 XCDs; give each XCD a contiguous range of logical blocks so rows that
// share density history share an L2.  A bijection when nblocks % 8 == 0.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int per = (nblocks + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// Local sum of lags m0 <= m < m1 (m0 = 1 or 2 for the right-hand side, 0 for
// the derivative sums of the gradient; m1 = NQ, or 2 for the lag-1 part), plus
// addin[j] when addin is not NULL, one row per wavefront.  The row's packed weights
// are one block per lag m (sources a_m .. a_m + c_m - 1 of its neighbour list,
// at offset off_m within the row).  Lane m loads lag m's (a, c, off); the
// wavefront then works as four groups of 16 lanes, group g on lag mb + g of
// the current quad of lags: each group streams one contiguous block of
// weights and densities, two consecutive elements per lane and load (16-byte
// loads, 256 bytes per group), eight elements per lane with every load issued
// before use.  A pair's second element may lie one past the block (its value
// is dropped; the packed arrays carry two spare elements) or, for the
// densities, wrap to source 0.
constexpr int kMaxNQ = 64;
// two consecutive doubles, 8-byte aligned (one 16-byte load)
typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));

// G lanes per lag (16 by default; 8 or 4 for rows whose lag blocks are
// short: 64 / G lags per trip, 8 G elements per lane group and trip).
template <int G = 16>
__device__ __forceinline__ void k_local_rhs_body(int M, int NQ, int NH, int64_t L, int m0, int m1,
            const int* __restrict__ nb_start, const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx,
            const double* __restrict__ Qc, const double* __restrict__ hist, const double* __restrict__ addin,
            double* __restrict__ loc, int bid, double* __restrict__ loc2 = nullptr, int nsplit = 1) {
  const int lane = threadIdx.x & 63;
  const int gw = bid * (blockDim.x >> 6) + (threadIdx.x >> 6);
  // nsplit > 1: nsplit wavefronts per row, part q on the q-th of nsplit equal
  // shares of the row's trips over lag groups (64 / G lags per trip); part 0
  // into loc (plus addin), part q > 0 into loc2[(q - 1) M + j], so each walks
  // a share of the row's lag blocks
  int j = gw;
  if (nsplit > 1) {
    j = gw / nsplit;
    const int part = gw - j * nsplit;
    const int nt = (m1 - m0 + 64 / G - 1) / (64 / G);
    const int a = m0 + (part * nt / nsplit) * (64 / G);
    m1 = min(m1, m0 + ((part + 1) * nt / nsplit) * (64 / G));
    m0 = a;
    if (part > 0) {
      loc = loc2 + (int64_t)(part - 1) * M;
      addin = nullptr;
    }
  }
  if (j >= M) return;   // no block-level barrier in this kernel
  const int st = nb_start[j];
  uint2 mine = make_uint2(0u, 0u);
  if (lane >= m0 && lane < m1) mine = acx[(int64_t)j * NQ + lane];
  const double* __restrict__ q = Qc + rowbase[j];
  const int grp = lane / G, gl = lane % G;
  double acc0 = 0.0, acc1 = 0.0;
  for (int mb = m0; mb < m1; mb += 64 / G) {
    const int m = mb + grp;
    const int src = m < 64 ? m : 0;
    const unsigned vx = __shfl(mine.x, src, 64), vy = __shfl(mine.y, src, 64);
    const int c = m < m1 ? (int)(vx >> 16) : 0;
    const double* __restrict__ qp = q + vy;
    const double* __restrict__ hp = hist + (int64_t)mod_slot(L - m, NH) * M;
    int l0 = st + (int)(vx & 0xffff);
    if (l0 >= M) l0 -= M;
    for (int i0 = 0; i0 < c; i0 += 8 * G) {
      d2u qv[4], hv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 2 * gl + 2 * G * u;
        qv[u] = d2u{0.0, 0.0};
        hv[u] = d2u{0.0, 0.0};
        if (i < c) {
          int la = l0 + i;
          if (la >= M) la -= M;
          qv[u] = *(const d2u*)(qp + i);
          if (la + 1 < M) {
            hv[u] = *(const d2u*)(hp + la);
          } else {
            hv[u].x = hp[la];
            hv[u].y = hp[0];
          }
          if (i + 1 >= c) {
            qv[u].y = 0.0;
            hv[u].y = 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc0 = fma(qv[u].x, hv[u].x, acc0);
        acc1 = fma(qv[u].y, hv[u].y, acc1);
      }
    }
  }
  const double accs = wave_sum(acc0 + acc1);
  if (lane == 0) loc[j] = addin ? addin[j] + accs : accs;
}

__global__ void __launch_bounds__(256)
k_local_rhs(int M, int NQ, int NH, int64_t L, int m0, int m1, const int* __restrict__ nb_start,
            const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx, const double* __restrict__ Qc,
            const double* __restrict__ hist, const double* __restrict__ addin, double* __restrict__ loc,
            double* __restrict__ loc2, int nsplit) {
  k_local_rhs_body(M, NQ, NH, L, m0, m1, nb_start, rowbase, acx, Qc, hist, addin, loc,
                   xcd_block(blockIdx.x, gridDim.x), loc2, nsplit);
}

// The same for rows with short lag blocks (8 or 4 lanes per lag).
__global__ void __launch_bounds__(256)
k_local_rhs_g8(int M, int NQ, int NH, int64_t L, int m0, int m1, const int* __restrict__ nb_start,
               const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx, const double* __restrict__ Qc,
               const double* __restrict__ hist, const double* __restrict__ addin, double* __restrict__ loc) {
  k_local_rhs_body<8>(M, NQ, NH, L, m0, m1, nb_start, rowbase, acx, Qc, hist, addin, loc,
                      xcd_block(blockIdx.x, gridDim.x));
}

__global__ void __launch_bounds__(256)
k_local_rhs_g4(int M, int NQ, int NH, int64_t L, int m0, int m1, const int* __restrict__ nb_start,
               const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx, const double* __restrict__ Qc,
               const double* __restrict__ hist, const double* __restrict__ addin, double* __restrict__ loc) {
  k_local_rhs_body<4>(M, NQ, NH, L, m0, m1, nb_start, rowbase, acx, Qc, hist, addin, loc,
                      xcd_block(blockIdx.x, gridDim.x));
}

// The lag-1 part of the right-hand side local sum added to the lags >= 2 part
// (which depends only on levels before L - 1, so it can be computed while
// level L - 1 is still being solved).  A row's lag-1 block is short (pairs
// closer than about p/2 dt), so 16 lanes take a row, two consecutive elements
// per lane and load as in k_local_rhs, and a wavefront takes four rows.
__global__ void __launch_bounds__(256)
k_local_lag1(int M, int NQ, int NH, int64_t L, const int* __restrict__ nb_start, const int64_t* __restrict__ rowbase,
             const uint2* __restrict__ acx, const double* __restrict__ Qc, const double* __restrict__ hist,
             const double* __restrict__ addin, const double* __restrict__ addin2, int nadd2,
             double* __restrict__ loc) {
  const int gl = threadIdx.x & 15;
  const int j = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 4) + (threadIdx.x >> 4);
  if (j >= M) return;   // no barrier; the reduction below stays inside the row's 16 lanes
  const uint2 v = acx[(int64_t)j * NQ + 1];
  const int c = (int)(v.x >> 16);
  const double* __restrict__ qp = Qc + rowbase[j] + v.y;
  const double* __restrict__ hp = hist + (int64_t)mod_slot(L - 1, NH) * M;
  int l0 = nb_start[j] + (int)(v.x & 0xffff);
  if (l0 >= M) l0 -= M;
  double acc0 = 0.0, acc1 = 0.0;
  for (int i0 = 0; i0 < c; i0 += 128) {
    d2u qv[4], hv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + 2 * gl + 32 * u;
      qv[u] = d2u{0.0, 0.0};
      hv[u] = d2u{0.0, 0.0};
      if (i < c) {
        int la = l0 + i;
        if (la >= M) la -= M;
        qv[u] = *(const d2u*)(qp + i);
        if (la + 1 < M) {
          hv[u] = *(const d2u*)(hp + la);
        } else {
          hv[u].x = hp[la];
          hv[u].y = hp[0];
        }
        if (i + 1 >= c) {
          qv[u].y = 0.0;
          hv[u].y = 0.0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc0 = fma(qv[u].x, hv[u].x, acc0);
      acc1 = fma(qv[u].y, hv[u].y, acc1);
    }
  }
  double sum = acc0 + acc1;
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (gl == 0) {
    double a = addin[j];
    for (int q = 0; q < nadd2; ++q) a += addin2[(int64_t)q * M + j];
    loc[j] = a + sum;
  }
}

// The gradient pass's two signed derivative local sums (lags 0 .. NQ - 1) in
// one stream of the derivative weights: out1 from levels held in a linear
// buffer (row r1 - m for lag m: the forward densities of the segment and the
// NQ - 1 levels before it), out2 from a density ring (slot L2 - m mod NH: the
// adjoint state).  Same row layout and loads as k_local_rhs_body.
__global__ void __launch_bounds__(256)
k_local_deriv2(int M, int NQ, int NH, const int* __restrict__ nb_start, const int64_t* __restrict__ rowbase,
               const uint2* __restrict__ acx, const double* __restrict__ Qc, const double* __restrict__ h1, int64_t r1,
               const double* __restrict__ h2, int64_t L2, double* __restrict__ out1, double* __restrict__ out2) {
  const int lane = threadIdx.x & 63;
  const int j = xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= M) return;   // no block-level barrier in this kernel
  const int st = nb_start[j];
  uint2 mine = make_uint2(0u, 0u);
  if (lane < NQ) mine = acx[(int64_t)j * NQ + lane];
  const double* __restrict__ q = Qc + rowbase[j];
  const int grp = lane >> 4, gl = lane & 15;
  double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
  for (int mb = 0; mb < NQ; mb += 4) {
    const int m = mb + grp;
    const int src = m < 64 ? m : 0;
    const unsigned vx = __shfl(mine.x, src, 64), vy = __shfl(mine.y, src, 64);
    const int c = m < NQ ? (int)(vx >> 16) : 0;
    const double* __restrict__ qp = q + vy;
    const double* __restrict__ hp1 = h1 + (r1 - (m < NQ ? m : 0)) * M;
    const double* __restrict__ hp2 = h2 + (int64_t)mod_slot(L2 - m, NH) * M;
    int l0 = st + (int)(vx & 0xffff);
    if (l0 >= M) l0 -= M;
    for (int i0 = 0; i0 < c; i0 += 128) {
      d2u qv[4], hv[4], gv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 2 * gl + 32 * u;
        qv[u] = d2u{0.0, 0.0};
        hv[u] = d2u{0.0, 0.0};
        gv[u] = d2u{0.0, 0.0};
        if (i < c) {
          int la = l0 + i;
          if (la >= M) la -= M;
          qv[u] = *(const d2u*)(qp + i);
          if (la + 1 < M) {
            hv[u] = *(const d2u*)(hp1 + la);
            gv[u] = *(const d2u*)(hp2 + la);
          } else {
            hv[u].x = hp1[la];
            hv[u].y = hp1[0];
            gv[u].x = hp2[la];
            gv[u].y = hp2[0];
          }
          if (i + 1 >= c) {
            qv[u].y = 0.0;
            hv[u].y = 0.0;
            gv[u].y = 0.0;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a0 = fma(qv[u].x, hv[u].x, a0);
        a1 = fma(qv[u].y, hv[u].y, a1);
        b0 = fma(qv[u].x, gv[u].x, b0);
        b1 = fma(qv[u].y, gv[u].y, b1);
      }
    }
  }
  const double s1 = wave_sum(a0 + a1), s2 = wave_sum(b0 + b1);
  if (lane == 0) {
    out1[j] = s1;
    out2[j] = s2;
  }
}


// Local sum of lags m >= 1 with the weights evaluated on the fly, each
// unordered pair of springs once.  Q_m(d) depends on the distance alone
// (Section 4.1), so the pair (j, l) shares its quadrature nodes, node weights,
// stencils and interpolation weights between the two rows it feeds:
//   row j:  sum_i om_i(d) sum_r v_{i,r} sigma_l^{L-m0_i-r},
//   row l:  sum_i om_i(d) sum_r v_{i,r} sigma_j^{L-m0_i-r},
// with the P lags from m0_i = max(m_min, floor(s_i) - P/2 + 1) (lag 0 taken as
// 0: it belongs to the implicit solve) and the Lagrange weights v_{i,r} of
// those lags at u = s_i - m0_i (SymLagrange below).  Sources are taken in
// sorted order: row j walks its upper
// range, the springs from j (itself, once) up to the first one beyond delta
// (unwrapped: periodic ranges continue past M - 1 at 0).  Every unordered pair
// lies in exactly one upper range because delta < pi.
// A block holds kOtfRows consecutive rows (one wavefront each); the union of
// their upper ranges is walked in chunks of kOtfChunk sources whose histories
// (lags 0..NQ-1, lag 0 zero) are staged in LDS, beside the rows' own.  Row j's
// sum goes to rowacc[j]; the column sums (row l's terms) are added over the
// block's wavefronts in LDS in a fixed order and written to
// part[part_off[b] + (u - j0)] for the block's unwrapped source u;
// k_local_otf_reduce adds them up per row.
// Lagrange weights of the P equispaced stencil lags in the centred variable
// y = u - (P-1)/2, whose nodes pair up as -a_j, +a_j, a_j = j + 1/2
// (j = 0..P/2-1; lag r < P/2 and lag P-1-r share j = P/2-1-r):
//   v_r = lambda_r (y - a_j) Q_j,   v_{P-1-r} = -lambda_r (y + a_j) Q_j,
//   Q_j = prod_{i != j} (y^2 - a_i^2),   lambda_r = (-1)^{P-1-r} / (r! (P-1-r)!),
// Q_j as products of a prefix and a suffix over i.  Every constant is a
// scalar operand of its instruction (one per instruction); the -a_j^2 are
// held in scalar registers by the caller (as immediates the compiler would
// rebuild them in vector registers at every node).
template <int P>
struct SymLagrange {
  static constexpr int H = P / 2;
  static constexpr double a(int j) { return j + 0.5; }
  struct Squares {
    double na2[H];
    __device__ __forceinline__ void init() {
#pragma unroll
      for (int j = 0; j < H; ++j) {
        na2[j] = -a(j) * a(j);
        asm volatile("" : "+s"(na2[j]));
      }
    }
  };
  static constexpr double lambda(int r) {
    double f = 1.0;
    for (int k = 2; k <= r; ++k) f *= k;
    for (int k = 2; k <= P - 1 - r; ++k) f *= k;
    return ((P - 1 - r) % 2 ? -1.0 : 1.0) / f;
  }
  __device__ __forceinline__ static void weights(double y, const Squares& sq, double (&w)[P]) {
    double e[H], pre[H], suf[H];
#pragma unroll
    for (int j = 0; j < H; ++j) e[j] = fma(y, y, sq.na2[j]);
    pre[0] = 1.0;
#pragma unroll
    for (int j = 1; j < H; ++j) pre[j] = pre[j - 1] * e[j - 1];
    suf[H - 1] = 1.0;
#pragma unroll
    for (int j = H - 2; j >= 0; --j) suf[j] = suf[j + 1] * e[j + 1];
#pragma unroll
    for (int r = 0; r < H; ++r) {
      const int j = H - 1 - r;
      const double t = lambda(r) * (pre[j] * suf[j]);
      const double ta = t * a(j);
      w[r] = fma(t, y, -ta);
      w[P - 1 - r] = fma(-t, y, -ta);
    }
  }
};

template <int P>
__device__ __forceinline__ void sym_node(double Dm, double span, int mmin, double na_q, double nw_q,
                                         const double* __restrict__ tab, double Wd, double pw,
                                         const double* __restrict__ sgk, const double* __restrict__ rh,
                                         const typename SymLagrange<P>::Squares& sq, double& acc_a,
                                         double& acc_c) {
  const double s = fma(Dm, na_q, Wd);         // W - (W - D)(1 + z_q)/2, in [0, W]
  // window piece: pc covers s in [pc, pc + 1) / pw, its polynomial in the
  // local variable x = v - pc (coefficients loaded here and used last, so the
  // loads overlap the interpolation).  v = pw W (s = W, only where the pair's
  // span rounds to 0) takes the last piece at x = 0, a weight-zero node.
  const double v = s * pw;
  unsigned pc = (unsigned)v;
  pc = pc >= (unsigned)kPhiPieces ? kPhiPieces - 1 : pc;
  const double* c = tab + pc * (kPhiDeg + 1);
  double cf[kPhiDeg + 1];
#pragma unroll
  for (int k = 0; k <= kPhiDeg; ++k) cf[k] = c[k];
  const double x = __builtin_amdgcn_fract(v);
  // stencil start max(mmin, floor(s) - P/2 + 1) (s >= 0: truncation is the
  // floor); s rounds to W only for d within an ulp of delta (zero weight):
  // the upper clamp keeps the stencil inside lags 0 .. W + P/2 - 1
  const int mtop = (int)Wd - P / 2;
  int m0;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(m0) : "v"((int)s - P / 2 + 1), "v"(mmin), "s"(mtop));
  const double* sp = sgk + m0 * kOtfChunk;
  const double* rp = rh + m0;
  double fa[P], fc[P];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    fa[r] = sp[r * kOtfChunk];
    fc[r] = rp[r];
  }
  double w[P];
  SymLagrange<P>::weights(s - (m0 + 0.5 * (P - 1)), sq, w);
  double pa = 0.0, pcl = 0.0;
#pragma unroll
  for (int r = 0; r < P; ++r) {
    pa = fma(w[r], fa[r], pa);
    pcl = fma(w[r], fc[r], pcl);
  }
  double ph = cf[kPhiDeg];
#pragma unroll
  for (int k = kPhiDeg - 1; k >= 0; --k) ph = fma(ph, x, cf[k]);
  const double om = span * nw_q * (1.0 - ph);
  acc_a = fma(om, pa, acc_a);
  acc_c = fma(om, pcl, acc_c);
}

template <int P>
__device__ __forceinline__ void k_local_otf_sym_body(int M, int NH, int NQ, int64_t L, const int* __restrict__ up_end,
                                                     const int* __restrict__ blk_end,
                                                     const int64_t* __restrict__ part_off,
                                                     const double* __restrict__ xs, const double* __restrict__ hist,
                                                     int periodic, double dt, double delta, int W, int ngl,
                                                     const double* __restrict__ na, const double* __restrict__ nw,
                                                     const double* __restrict__ phitab, double* __restrict__ rowacc,
                                                     double* __restrict__ part, int b) {
  extern __shared__ double sg[];                              // [NQ][kOtfChunk], then [kOtfRows][kOtfChunk]
  __shared__ double tab[kPhiPieces * (kPhiDeg + 1)];
  __shared__ double rh[kOtfRows][kMaxOtfLags + 1];
  __shared__ int64_t slot[kMaxOtfLags + 1];                   // row offset of lag m's density level
  double* colp = sg + (size_t)NQ * kOtfChunk;                 // per-wavefront column sums of a chunk
  for (int i = threadIdx.x; i < kPhiPieces * (kPhiDeg + 1); i += blockDim.x) tab[i] = phitab[i];
  for (int m = threadIdx.x; m < NQ; m += blockDim.x) slot[m] = (int64_t)mod_slot(L - m, NH) * M;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j0 = b * kOtfRows;
  const int j = j0 + wv;
  const bool row = j < M;
  __syncthreads();
  for (int e = threadIdx.x; e < kOtfRows * NQ; e += blockDim.x) {
    const int w = e / NQ, m = e - w * NQ;
    rh[w][m] = (m >= 1 && j0 + w < M) ? hist[slot[m] + (j0 + w)] : 0.0;
  }
  for (int k = threadIdx.x; k < kOtfChunk; k += blockDim.x) sg[k] = 0.0;   // lag 0
  const long long uend = blk_end[b];                          // unwrapped end of the block's sources
  const long long my1 = row ? up_end[j] : j;                  // row's upper range [j, my1)
  const double xa = row ? xs[j] : 0.0;
  const double Wd = (double)W;
  const double pw = (double)kPhiPieces / Wd;
  const int64_t pbase = part_off[b];
  typename SymLagrange<P>::Squares sq;
  sq.init();
  double acc = 0.0;
  for (long long cb = j0; cb < uend; cb += kOtfChunk) {
    __syncthreads();   // the previous chunk is no longer read
    for (int e = threadIdx.x; e < (NQ - 1) * kOtfChunk; e += blockDim.x) {
      const int m = e / kOtfChunk + 1, k = e - (m - 1) * kOtfChunk;
      const long long u = cb + k;                             // < 2M
      double v = 0.0;
      if (u < uend) v = hist[slot[m] + (u < M ? u : u - M)];
      sg[m * kOtfChunk + k] = v;
    }
    for (int e = threadIdx.x; e < kOtfRows * kOtfChunk; e += blockDim.x) colp[e] = 0.0;
    __syncthreads();
    const long long a0 = (long long)j > cb ? (long long)j : cb;
    const long long a1 = my1 < cb + kOtfChunk ? my1 : cb + kOtfChunk;
    for (long long ua = a0 + lane; ua < a1; ua += 64) {
      double d = fabs(xa - xs[ua < M ? (int)ua : (int)(ua - M)]);
      if (periodic && d > kPi) d = kTwoPi - d;
      const bool on = d < delta;
      const int k = (int)(ua - cb);
      const double Dm = on ? d / dt - Wd : -0.5 * Wd;    // off: D = W/2, nodes inside (0, W), zero weight
      const int mmin = (on && d < dt) ? 0 : 1;
      const double span = on ? delta - d : 0.0;
      double pa = 0.0, pcol = 0.0;
      for (int q = 0; q < ngl; ++q) sym_node<P>(Dm, span, mmin, na[q], nw[q], tab, Wd, pw, sg + k, rh[wv], sq, pa, pcol);
      acc += pa;
      if (ua != (long long)j) colp[wv * kOtfChunk + k] = pcol;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kOtfChunk; k += blockDim.x) {
      const long long u = cb + k;
      if (u < uend) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < kOtfRows; ++w) sum += colp[w * kOtfChunk + k];
        part[pbase + (u - j0)] = sum;
      }
    }
  }
  acc = wave_sum(acc);
  if (row && lane == 0) rowacc[j] = acc;
}

template <int P>
__global__ void __launch_bounds__(1024)
k_local_otf_sym(int M, int NH, int NQ, int64_t L, const int* __restrict__ up_end, const int* __restrict__ blk_end,
                const int64_t* __restrict__ part_off, int nblk_rows, const double* __restrict__ xs,
                const double* __restrict__ hist, int periodic, double dt, double delta, int W, int ngl,
                const double* __restrict__ na, const double* __restrict__ nw, const double* __restrict__ phitab,
                double* __restrict__ rowacc, double* __restrict__ part) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= nblk_rows) return;                                 // padding block: nothing to do
  k_local_otf_sym_body<P>(M, NH, NQ, L, up_end, blk_end, part_off, xs, hist, periodic, dt, delta, W, ngl, na, nw,
                          phitab, rowacc, part, b);
}

// Row l's total of the symmetric local sum: its own upper-range sum plus the
// column sums that the blocks covering l wrote for it (blocks at or below
// l's own whose source range reaches l, and in the periodic box the blocks
// whose range wraps past M - 1 to l + M), in a fixed order; scaled per row.
__device__ __forceinline__ void k_local_otf_reduce_body(int M, int nblk_rows, int periodic,
                                                        const int* __restrict__ blk_end,
                                                        const int64_t* __restrict__ part_off,
                                                        const double* __restrict__ rowacc,
                                                        const double* __restrict__ part,
                                                        const double* __restrict__ scale, double* __restrict__ out,
                                                        int bid) {
  const int l = bid * 256 + threadIdx.x;
  if (l >= M) return;
  double acc = rowacc[l];
  for (int b = l / kOtfRows; b >= 0 && blk_end[b] > l; --b) acc += part[part_off[b] + (l - b * kOtfRows)];
  if (periodic) {
    const long long lw = (long long)l + M;
    for (int b = nblk_rows - 1; b >= 0 && blk_end[b] > lw; --b) acc += part[part_off[b] + (lw - (long long)b * kOtfRows)];
  }
  out[l] = scale[l] * acc;
}

__global__ void __launch_bounds__(256)
k_local_otf_reduce(int M, int nblk_rows, int periodic, const int* __restrict__ blk_end,
                   const int64_t* __restrict__ part_off, const double* __restrict__ rowacc,
                   const double* __restrict__ part, const double* __restrict__ scale, double* __restrict__ out) {
  k_local_otf_reduce_body(M, nblk_rows, periodic, blk_end, part_off, rowacc, part, scale, out, blockIdx.x);
}

#define WFP_OTFS_INST(PP)                                                                                      \
  template __global__ void k_local_otf_sym<PP>(int, int, int, int64_t, const int*, const int*, const int64_t*, \
                                               int, const double*, const double*, int, double, double, int, int, \
                                               const double*, const double*, const double*, double*, double*);
WFP_OTFS_INST(2)
WFP_OTFS_INST(4)
WFP_OTFS_INST(6)
WFP_OTFS_INST(8)
WFP_OTFS_INST(10)
WFP_OTFS_INST(12)
#undef WFP_OTFS_INST

// First lag m in [m0, NQ) whose run of sources reaches index i0 of the upper
// range (c_m > i0), NQ if none.  The runs are prefixes whose length does not
// decrease with the lag (a source carries the lags from its stencil's lowest
// one up, and that grows with the distance), so the lags below it contribute
// only zeros for sources i0 and beyond.
__device__ __forceinline__ int first_lag_reaching(const uint2* __restrict__ cw, int m0, int NQ, int i0) {
  int lo = m0, hi = NQ;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int)cw[mid].x > i0) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

// Local sum of lags m >= mfirst (1, or 2 with the lag-1 part added by
// k_local_sym_lag1) from stored weights, each unordered pair once.
// One wavefront per row j walks its upper range [j, up_end[j]) (unwrapped:
// periodic ranges continue past M - 1 at 0), each lane over SPL consecutive
// sources (2: one 16-byte load of each pair's weights and densities, for long
// ranges; 1: every lane busy on short ones), lags in groups of 8 / SPL with
// every load of a group issued before its use.  Row j's
// weights are one run per lag m over the first c_jm sources of the range
// (those whose stencils reach lag m: a prefix, as the distance grows along the
// range), at Qs[rb[j] + o_jm + i], sacx[j NQ + m] = (c_jm, o_jm), unscaled.
// The row's own sum sum_m sum_i Q sigma_l goes to rowacc[j]; each pair's
// column term sum_m Q sigma_j^{L-m} (row l's share) to colpart[upb[j] + i]
// (0 for the row itself); k_local_sym_reduce adds them up per row.
template <int SPL>
__device__ __forceinline__ void k_local_sym_rows_body(int M, int NH, int NQ, int64_t L, int mfirst,
                                                      const int* __restrict__ up_end, const double* __restrict__ hist,
                                                      const int64_t* __restrict__ rb, const uint2* __restrict__ sacx,
                                                      const double* __restrict__ Qs, const int64_t* __restrict__ upb,
                                                      double* __restrict__ rowacc, double* __restrict__ colpart,
                                                      int b) {
  __shared__ double rv[4][kMaxOtfLags + 1];                   // each row's own history, lags 0 .. NQ - 1
  __shared__ uint2 cw[4][kMaxOtfLags + 1];
  __shared__ int64_t slot[kMaxOtfLags + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = b * 4 + wv;
  for (int m = threadIdx.x; m < NQ; m += blockDim.x) slot[m] = (int64_t)mod_slot(L - m, NH) * M;
  __syncthreads();
  for (int e = threadIdx.x; e < 4 * NQ; e += blockDim.x) {
    const int w = e / NQ, m = e - w * NQ;
    const int jr = b * 4 + w;
    const bool ok = m >= 1 && jr < M;
    rv[w][m] = ok ? hist[slot[m] + jr] : 0.0;
    cw[w][m] = ok ? sacx[(int64_t)jr * NQ + m] : make_uint2(0u, 0u);
  }
  __syncthreads();
  if (j >= M) return;                                         // no barrier below
  const int n = up_end[j] - j;
  const double* __restrict__ qrow = Qs + rb[j];
  double* __restrict__ cp = colpart + upb[j];
  if constexpr (SPL == 1) {
    double acc = 0.0;
    for (int i0 = 0; i0 < n; i0 += 64) {
      const int i = i0 + lane;
      const bool in = i < n;
      int l = j + i;
      if (l >= M) l -= M;
      double pc = 0.0;
      for (int mb = first_lag_reaching(cw[wv], mfirst, NQ, i0); mb < NQ; mb += 8) {
        double w[8], h[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int m = mb + r;
          const uint2 c = m < NQ ? cw[wv][m] : make_uint2(0u, 0u);
          const bool on = in && i < (int)c.x;
          w[r] = on ? qrow[c.y + i] : 0.0;
          h[r] = on ? hist[slot[m] + l] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int m = mb + r;
          if (m < NQ) {
            acc = fma(w[r], h[r], acc);
            pc = fma(w[r], rv[wv][m], pc);
          }
        }
      }
      if (in) cp[i] = i == 0 ? 0.0 : pc;
    }
    acc = wave_sum(acc);
    if (lane == 0) rowacc[j] = acc;
  } else {
    double acc0 = 0.0, acc1 = 0.0;
    for (int i0 = 0; i0 < n; i0 += 128) {
      // sources i and i + 1 of the range, one 16-byte load of each pair's
      // weights and densities (a weight one past a run is read and dropped:
      // the packed array carries two spare elements; a density pair that would
      // run past source M - 1 continues at source 0)
      const int i = i0 + 2 * lane;
      const bool in0 = i < n, in1 = i + 1 < n;
      int l = j + i;
      if (l >= M) l -= M;
      const bool adj = l + 1 < M;
      double pc0 = 0.0, pc1 = 0.0;
      for (int mb = first_lag_reaching(cw[wv], mfirst, NQ, i0); mb < NQ; mb += 4) {
        d2u w[4], h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mb + r;
          const uint2 c = m < NQ ? cw[wv][m] : make_uint2(0u, 0u);
          w[r] = d2u{0.0, 0.0};
          h[r] = d2u{0.0, 0.0};
          if (in0 && i < (int)c.x) {
            const double* __restrict__ hp = hist + slot[m];
            w[r] = *(const d2u*)(qrow + c.y + i);
            if (adj) {
              h[r] = *(const d2u*)(hp + l);
            } else {
              h[r].x = hp[l];
              h[r].y = hp[0];
            }
            if (!(in1 && i + 1 < (int)c.x)) {
              w[r].y = 0.0;
              h[r].y = 0.0;
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mb + r;
          if (m < NQ) {
            acc0 = fma(w[r].x, h[r].x, acc0);
            acc1 = fma(w[r].y, h[r].y, acc1);
            pc0 = fma(w[r].x, rv[wv][m], pc0);
            pc1 = fma(w[r].y, rv[wv][m], pc1);
          }
        }
      }
      if (in0) cp[i] = i == 0 ? 0.0 : pc0;
      if (in1) cp[i + 1] = pc1;
    }
    const double acc = wave_sum(acc0 + acc1);
    if (lane == 0) rowacc[j] = acc;
  }
}

template <int SPL>
__global__ void __launch_bounds__(256)
k_local_sym_rows(int M, int NH, int NQ, int64_t L, int mfirst, const int* __restrict__ up_end,
                 const double* __restrict__ hist, const int64_t* __restrict__ rb, const uint2* __restrict__ sacx,
                 const double* __restrict__ Qs, const int64_t* __restrict__ upb, double* __restrict__ rowacc,
                 double* __restrict__ colpart) {
  k_local_sym_rows_body<SPL>(M, NH, NQ, L, mfirst, up_end, hist, rb, sacx, Qs, upb, rowacc, colpart,
                             xcd_block(blockIdx.x, gridDim.x));
}

// The gradient pass's two signed derivative local sums (lags 0 .. NQ - 1)
// from derivative weights stored once per unordered pair.  Row j's weight
// for the source l of its upper range is w = (1/2) dQ_m/dd sign(x_j - x_l),
// which changes sign with the pair's order, so row l's share is -w times row
// j's values.  Values for the first sum from a linear buffer (row r1 - m for
// lag m: the forward densities of the segment and the NQ - 1 levels before
// it), for the second from a ring (slot L2 - m mod NH: the adjoint state).
// One wavefront per row, SPL sources per lane, as in k_local_sym_rows; each
// pair's column terms, negated, go to col1 / col2[upb[j] + i] (0 for the row
// itself), and k_local_sym_reduce adds them up per row.
template <int SPL>
__global__ void __launch_bounds__(256)
k_local_sym_deriv2(int M, int NQ, int NH, const int* __restrict__ up_end, const double* __restrict__ h1, int64_t r1,
                   const double* __restrict__ h2, int64_t L2, const int64_t* __restrict__ rb,
                   const uint2* __restrict__ sacx, const double* __restrict__ Qs, const int64_t* __restrict__ upb,
                   double* __restrict__ row1, double* __restrict__ row2, double* __restrict__ col1,
                   double* __restrict__ col2) {
  __shared__ double rv1[4][kMaxOtfLags + 1], rv2[4][kMaxOtfLags + 1];   // each row's own values, lags 0 .. NQ - 1
  __shared__ uint2 cw[4][kMaxOtfLags + 1];
  __shared__ int64_t s1[kMaxOtfLags + 1], s2[kMaxOtfLags + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nb = gridDim.x;
  const int j = xcd_block(blockIdx.x, nb) * 4 + wv;
  for (int m = threadIdx.x; m < NQ; m += blockDim.x) {
    s1[m] = (r1 - m) * M;
    s2[m] = (int64_t)mod_slot(L2 - m, NH) * M;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 4 * NQ; e += blockDim.x) {
    const int w = e / NQ, m = e - w * NQ;
    const int jr = xcd_block(blockIdx.x, nb) * 4 + w;
    const bool ok = jr < M;
    rv1[w][m] = ok ? h1[s1[m] + jr] : 0.0;
    rv2[w][m] = ok ? h2[s2[m] + jr] : 0.0;
    cw[w][m] = ok ? sacx[(int64_t)jr * NQ + m] : make_uint2(0u, 0u);
  }
  __syncthreads();
  if (j >= M) return;                                         // no barrier below
  const int n = up_end[j] - j;
  const double* __restrict__ qrow = Qs + rb[j];
  double* __restrict__ cp1 = col1 + upb[j];
  double* __restrict__ cp2 = col2 + upb[j];
  if constexpr (SPL == 1) {
    double a1 = 0.0, a2 = 0.0;
    for (int i0 = 0; i0 < n; i0 += 64) {
      const int i = i0 + lane;
      const bool in = i < n;
      int l = j + i;
      if (l >= M) l -= M;
      double p1 = 0.0, p2 = 0.0;
      for (int mb = first_lag_reaching(cw[wv], 0, NQ, i0); mb < NQ; mb += 8) {
        double w[8], g1[8], g2[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int m = mb + r;
          const uint2 c = m < NQ ? cw[wv][m] : make_uint2(0u, 0u);
          const bool on = in && i < (int)c.x;
          w[r] = on ? qrow[c.y + i] : 0.0;
          g1[r] = on ? h1[s1[m] + l] : 0.0;
          g2[r] = on ? h2[s2[m] + l] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int m = mb + r;
          if (m < NQ) {
            a1 = fma(w[r], g1[r], a1);
            a2 = fma(w[r], g2[r], a2);
            p1 = fma(w[r], rv1[wv][m], p1);
            p2 = fma(w[r], rv2[wv][m], p2);
          }
        }
      }
      if (in) {
        cp1[i] = i == 0 ? 0.0 : -p1;
        cp2[i] = i == 0 ? 0.0 : -p2;
      }
    }
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    if (lane == 0) {
      row1[j] = a1;
      row2[j] = a2;
    }
  } else {
    double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int i0 = 0; i0 < n; i0 += 128) {
      // sources i and i + 1, 16-byte loads as in k_local_sym_rows
      const int i = i0 + 2 * lane;
      const bool in0 = i < n, in1 = i + 1 < n;
      int l = j + i;
      if (l >= M) l -= M;
      const bool adj = l + 1 < M;
      double p1 = 0.0, p2 = 0.0, q1 = 0.0, q2 = 0.0;
      for (int mb = first_lag_reaching(cw[wv], 0, NQ, i0); mb < NQ; mb += 4) {
        d2u w[4], g1[4], g2[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mb + r;
          const uint2 c = m < NQ ? cw[wv][m] : make_uint2(0u, 0u);
          w[r] = d2u{0.0, 0.0};
          g1[r] = d2u{0.0, 0.0};
          g2[r] = d2u{0.0, 0.0};
          if (in0 && i < (int)c.x) {
            const double* __restrict__ hp1 = h1 + s1[m];
            const double* __restrict__ hp2 = h2 + s2[m];
            w[r] = *(const d2u*)(qrow + c.y + i);
            if (adj) {
              g1[r] = *(const d2u*)(hp1 + l);
              g2[r] = *(const d2u*)(hp2 + l);
            } else {
              g1[r].x = hp1[l];
              g1[r].y = hp1[0];
              g2[r].x = hp2[l];
              g2[r].y = hp2[0];
            }
            if (!(in1 && i + 1 < (int)c.x)) {
              w[r].y = 0.0;
              g1[r].y = 0.0;
              g2[r].y = 0.0;
            }
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = mb + r;
          if (m < NQ) {
            a1 = fma(w[r].x, g1[r].x, a1);
            b1 = fma(w[r].y, g1[r].y, b1);
            a2 = fma(w[r].x, g2[r].x, a2);
            b2 = fma(w[r].y, g2[r].y, b2);
            p1 = fma(w[r].x, rv1[wv][m], p1);
            q1 = fma(w[r].y, rv1[wv][m], q1);
            p2 = fma(w[r].x, rv2[wv][m], p2);
            q2 = fma(w[r].y, rv2[wv][m], q2);
          }
        }
      }
      if (in0) {
        cp1[i] = i == 0 ? 0.0 : -p1;
        cp2[i] = i == 0 ? 0.0 : -p2;
      }
      if (in1) {
        cp1[i + 1] = -q1;
        cp2[i + 1] = -q2;
      }
    }
    const double s1sum = wave_sum(a1 + b1), s2sum = wave_sum(a2 + b2);
    if (lane == 0) {
      row1[j] = s1sum;
      row2[j] = s2sum;
    }
  }
}

template __global__ void k_local_sym_rows<1>(int, int, int, int64_t, int, const int*, const double*, const int64_t*,
                                             const uint2*, const double*, const int64_t*, double*, double*);
template __global__ void k_local_sym_rows<2>(int, int, int, int64_t, int, const int*, const double*, const int64_t*,
                                             const uint2*, const double*, const int64_t*, double*, double*);
template __global__ void k_local_sym_deriv2<1>(int, int, int, const int*, const double*, int64_t, const double*,
                                               int64_t, const int64_t*, const uint2*, const double*,
                                               const int64_t*, double*, double*, double*, double*);
template __global__ void k_local_sym_deriv2<2>(int, int, int, const int*, const double*, int64_t, const double*,
                                               int64_t, const int64_t*, const uint2*, const double*,
                                               const int64_t*, double*, double*, double*, double*);

// The gradient pass's two signed derivative local sums (lags 0 .. NQ - 1)
// with the weights evaluated on the fly, each unordered pair once.  For the
// pair (j, l) at distance d (Section 4.1),
//   Q_m(d) = sum_i om_i(d) v_{i,m}(s_i(d)),  om_i = (delta - d) (w_i/2) (1 - phi(s_i)),
//   s_i = W - (W - d/dt)(1 + z_i)/2,  ds_i/dd = (1 + z_i)/(2 dt),
// so dQ_m/dd = sum_i [ dom_i/dd v_{i,m} + om_i v'_{i,m} ds_i/dd ] with
//   dom_i/dd = (w_i/2) ( -(1 - phi(s_i)) - (delta - d) phi'(s_i) ds_i/dd )
// (phi' from the derivative of the window piece's polynomial, v' from the
// centred Lagrange form below).  Row j's weight for source l is
// (1/2) dQ_m/dd sign(x_j - x_l), which changes sign with the pair's order:
// row j adds it times the source's values, row l minus it times row j's.
// First sum from a linear buffer of levels (row r1 - m for lag m: the forward
// densities), second from a ring (slot L2 - m mod NH: the adjoint state);
// lag 0 holds the current level of each.  Blocks of kOtfRows rows walk the
// union of their upper ranges in chunks of kOtfDerivChunk sources, staged in
// LDS with both histories; the column terms are added over the block's
// wavefronts in a fixed order into part1 / part2, and k_local_otf_reduce adds
// them up per row.  The same pass forms the next adjoint level's explicit
// local sum, sum_{m >= 1} (1/2) Q_m(d) of the second history at lag m - 1
// (the adjoint state one level on), into row3 / part3: its weights om_i v_i
// come with the derivative ones, its operands are the loaded ones shifted by
// one lag plus lag m0 - 1 (zero below lag 0).
// c_r = a w_r(y) + b w_r'(y) and v_r = g w_r(y) for the centred Lagrange
// weights of the p-point stencil (the weights' form in SymLagrange,
// differentiated through the prefix and suffix products of the factors
// y^2 - a_k^2): one node's derivative weights, with a = d(omega)/dd and
// b = omega ds/dd, and its weights, with g = omega.
template <int P>
__device__ __forceinline__ void sym_lagrange_comb(double y, const typename SymLagrange<P>::Squares& sq, double a,
                                                  double b, double g, double (&c)[P], double (&v)[P]) {
  constexpr int H = P / 2;
  double e[H], pre[H], suf[H], dpre[H], dsuf[H];
  const double y2 = 2.0 * y;
#pragma unroll
  for (int j = 0; j < H; ++j) e[j] = fma(y, y, sq.na2[j]);
  pre[0] = 1.0;
  dpre[0] = 0.0;
#pragma unroll
  for (int j = 1; j < H; ++j) {
    pre[j] = pre[j - 1] * e[j - 1];
    dpre[j] = fma(dpre[j - 1], e[j - 1], pre[j - 1] * y2);
  }
  suf[H - 1] = 1.0;
  dsuf[H - 1] = 0.0;
#pragma unroll
  for (int j = H - 2; j >= 0; --j) {
    suf[j] = suf[j + 1] * e[j + 1];
    dsuf[j] = fma(dsuf[j + 1], e[j + 1], suf[j + 1] * y2);
  }
#pragma unroll
  for (int r = 0; r < H; ++r) {
    const int j = H - 1 - r;
    const double lam = SymLagrange<P>::lambda(r), aj = SymLagrange<P>::a(j);
    // w_r = t (y - a_j), w_{P-1-r} = -t (y + a_j); w' adds t' (y -+ a_j) +- t
    const double t = lam * (pre[j] * suf[j]);
    const double td = lam * fma(dpre[j], suf[j], pre[j] * dsuf[j]);
    const double T = fma(a, t, b * td), bt = b * t, gt = g * t;
    c[r] = fma(T, y - aj, bt);
    c[P - 1 - r] = -fma(T, y + aj, bt);
    v[r] = gt * (y - aj);
    v[P - 1 - r] = -gt * (y + aj);
  }
}

template <int P>
__global__ void __launch_bounds__(64 * kOtfRows)
k_local_otf_deriv2(int M, int NH, int NQ, const int* __restrict__ up_end, const int* __restrict__ blk_end,
                   const int64_t* __restrict__ part_off, int nblk_rows, const double* __restrict__ xs,
                   const double* __restrict__ h1, int64_t r1, const double* __restrict__ h2, int64_t L2,
                   int periodic, double dt, double delta, int W, int ngl, const double* __restrict__ na,
                   const double* __restrict__ nw, const double* __restrict__ phitab, double* __restrict__ row1,
                   double* __restrict__ row2, double* __restrict__ row3, double* __restrict__ part1,
                   double* __restrict__ part2, double* __restrict__ part3) {
  constexpr int CH = kOtfDerivChunk;
  // both histories side by side (one 16-byte read per stencil point):
  // [NQ][CH] pairs of the sources', then [kOtfRows][CH] x 3 column sums
  extern __shared__ double2 sd2[];
  __shared__ double tab[kPhiPieces * (kPhiDeg + 1)];
  __shared__ double2 rh[kOtfRows][kMaxOtfLags + 1];
  __shared__ int64_t sl1[kMaxOtfLags + 1], sl2[kMaxOtfLags + 1];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= nblk_rows) return;   // padding block: nothing to do (block-uniform)
  double2* sg = sd2;
  double* cp1 = (double*)(sd2 + (size_t)NQ * CH);
  double* cp2 = cp1 + (size_t)kOtfRows * CH;
  double* cp3 = cp2 + (size_t)kOtfRows * CH;
  const double* sgd = (const double*)sg;
  for (int i = threadIdx.x; i < kPhiPieces * (kPhiDeg + 1); i += blockDim.x) tab[i] = phitab[i];
  for (int m = threadIdx.x; m < NQ; m += blockDim.x) {
    sl1[m] = (r1 - m) * M;
    sl2[m] = (int64_t)mod_slot(L2 - m, NH) * M;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j0 = b * kOtfRows;
  const int j = j0 + wv;
  const bool row = j < M;
  __syncthreads();
  for (int e = threadIdx.x; e < kOtfRows * NQ; e += blockDim.x) {
    const int w = e / NQ, m = e - w * NQ;
    const bool ok = j0 + w < M;
    rh[w][m] = ok ? make_double2(h1[sl1[m] + (j0 + w)], h2[sl2[m] + (j0 + w)]) : make_double2(0.0, 0.0);
  }
  const long long uend = blk_end[b];
  const long long my1 = row ? up_end[j] : j;
  const double xa = row ? xs[j] : 0.0;
  const double Wd = (double)W;
  const double pw = (double)kPhiPieces / Wd;
  const int64_t pbase = part_off[b];
  typename SymLagrange<P>::Squares sq;
  sq.init();
  double acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  for (long long cb = j0; cb < uend; cb += CH) {
    __syncthreads();   // the previous chunk is no longer read
    for (int e = threadIdx.x; e < NQ * CH; e += blockDim.x) {
      const int m = e / CH, k = e - m * CH;
      const long long u = cb + k;   // < 2M
      double v1 = 0.0, v2 = 0.0;
      if (u < uend) {
        const int uu = (int)(u < M ? u : u - M);
        v1 = h1[sl1[m] + uu];
        v2 = h2[sl2[m] + uu];
      }
      sg[e] = make_double2(v1, v2);
    }
    for (int e = threadIdx.x; e < kOtfRows * CH; e += blockDim.x) {
      cp1[e] = 0.0;
      cp2[e] = 0.0;
      cp3[e] = 0.0;
    }
    __syncthreads();
    const long long a0 = (long long)j > cb ? (long long)j : cb;
    const long long a1 = my1 < cb + CH ? my1 : cb + CH;
    for (long long ua = a0 + lane; ua < a1; ua += 64) {
      const int l = ua < M ? (int)ua : (int)(ua - M);
      double y = xa - xs[l];
      if (periodic) y -= kTwoPi * rint(y * kInvTwoPi);
      const double d = fabs(y);
      const bool on = d < delta;
      const double f = on ? 0.5 * ((y > 0.0) ? 1.0 : ((y < 0.0) ? -1.0 : 0.0)) : 0.0;
      const int k = (int)(ua - cb);
      const double Dm = on ? d / dt - Wd : -0.5 * Wd;
      const int mmin = (on && d < dt) ? 0 : 1;
      const double span = on ? delta - d : 0.0;
      const int mtop = (int)Wd - P / 2;
      double s1 = 0.0, s2 = 0.0, t1 = 0.0, t2 = 0.0, s3 = 0.0, t3 = 0.0;
      for (int q = 0; q < ngl; ++q) {
        const double naq = na[q], nwq = nw[q];
        const double s = fma(Dm, naq, Wd);
        const double ds_dd = naq / dt;
        const double v = s * pw;
        unsigned pc = (unsigned)v;
        pc = pc >= (unsigned)kPhiPieces ? kPhiPieces - 1 : pc;
        const double* c = tab + pc * (kPhiDeg + 1);
        const double x = __builtin_amdgcn_fract(v);
        double ph = c[kPhiDeg], dph = 0.0;
#pragma unroll
        for (int kk = kPhiDeg - 1; kk >= 0; --kk) {
          dph = fma(dph, x, ph);
          ph = fma(ph, x, c[kk]);
        }
        int m0 = (int)s - P / 2 + 1;
        m0 = m0 < mmin ? mmin : (m0 > mtop ? mtop : m0);
        // d/dd [omega v_r(s)] = (d omega/dd) v_r + omega v_r' ds/dd
        const double om = span * nwq * (1.0 - ph);
        const double dom = nwq * (-(1.0 - ph) - span * (dph * pw) * ds_dd);
        double cw[P], vw[P];
        sym_lagrange_comb<P>(s - (m0 + 0.5 * (P - 1)), sq, dom, om * ds_dd, om, cw, vw);
        // the second history one lag down for the next level's sum: lag m0 - 1
        // (zero for m0 = 0, read at lag 0 to stay in bounds), then the loaded ones
        const int mp = m0 > 0 ? m0 - 1 : 0;
        double gp = sgd[2 * (mp * CH + k) + 1], op = rh[wv][mp].y;
        gp = m0 > 0 ? gp : 0.0;
        op = m0 > 0 ? op : 0.0;
#pragma unroll
        for (int r = 0; r < P; ++r) {
          const double2 g = sg[(m0 + r) * CH + k], o = rh[wv][m0 + r];
          s1 = fma(cw[r], g.x, s1);
          s2 = fma(cw[r], g.y, s2);
          t1 = fma(cw[r], o.x, t1);
          t2 = fma(cw[r], o.y, t2);
          s3 = fma(vw[r], gp, s3);
          t3 = fma(vw[r], op, t3);
          gp = g.y;
          op = o.y;
        }
      }
      acc1 = fma(f, s1, acc1);
      acc2 = fma(f, s2, acc2);
      acc3 += s3;
      if (ua != (long long)j) {
        cp1[wv * CH + k] = -f * t1;
        cp2[wv * CH + k] = -f * t2;
        cp3[wv * CH + k] = t3;
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < CH; k += blockDim.x) {
      const long long u = cb + k;
      if (u < uend) {
        double u1 = 0.0, u2 = 0.0, u3 = 0.0;
#pragma unroll
        for (int w = 0; w < kOtfRows; ++w) {
          u1 += cp1[w * CH + k];
          u2 += cp2[w * CH + k];
          u3 += cp3[w * CH + k];
        }
        part1[pbase + (u - j0)] = u1;
        part2[pbase + (u - j0)] = u2;
        part3[pbase + (u - j0)] = u3;
      }
    }
  }
  acc1 = wave_sum(acc1);
  acc2 = wave_sum(acc2);
  acc3 = wave_sum(acc3);
  if (row && lane == 0) {
    row1[j] = acc1;
    row2[j] = acc2;
    row3[j] = acc3;
  }
}

#define WFP_OTFD_INST(PP)                                                                                       \
  template __global__ void k_local_otf_deriv2<PP>(int, int, int, const int*, const int*, const int64_t*, int,     \
                                                  const double*, const double*, int64_t, const double*, int64_t,  \
                                                  int, double, double, int, int, const double*, const double*,    \
                                                  const double*, double*, double*, double*, double*, double*,     \
                                                  double*);
WFP_OTFD_INST(2)
WFP_OTFD_INST(4)
WFP_OTFD_INST(6)
WFP_OTFD_INST(8)
WFP_OTFD_INST(10)
WFP_OTFD_INST(12)
#undef WFP_OTFD_INST

// Row l's total of the pair-once stored local sum: its own sum plus the column
// terms of the rows whose upper range covers it: rows cov[l].x .. l - 1 (up_end
// is non-decreasing, so they are consecutive) and, in the periodic box, rows
// cov[l].y .. M - 1 whose range wraps to l + M; scaled per row.  A workgroup
// takes 64 consecutive rows, one per lane, so that a covering row's terms for
// them are consecutive in its block of colpart (one coalesced load per
// covering row).  The union of the 64 rows' covering rows is cut into 16
// consecutive parts, one per wavefront, each adding its part in order; the
// partial sums are then added in a fixed order.
__device__ __forceinline__ void k_local_sym_reduce_body(int M, const int2* __restrict__ cov,
                                                        const int64_t* __restrict__ upb,
                                                        const double* __restrict__ rowacc,
                                                        const double* __restrict__ colpart,
                                                        const double* __restrict__ scale, double* __restrict__ out,
                                                        int bid) {
  __shared__ double part[kReduceWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int l0 = bid * 64;
  const int l = l0 + lane;
  const bool act = l < M;
  const int2 c = act ? cov[l] : make_int2(M, M);
  // cov[l].x and cov[l].y do not decrease with l: the block's covering rows
  // below are cov[l0].x .. lend - 2, its wrapping rows cov[l0].y .. M - 1
  const int lend = min(l0 + 64, M);
  const int2 c0 = cov[l0];
  const int a0 = c0.x, n1 = max(lend - 1 - a0, 0);
  const int b0 = c0.y, n2 = max(M - b0, 0);
  const int ntot = n1 + n2;
  const int q0 = (int)((int64_t)wv * ntot / kReduceWaves), q1 = (int)((int64_t)(wv + 1) * ntot / kReduceWaves);
  double acc = 0.0;
  for (int q = q0; q < q1; q += 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = q + u;
      v[u] = 0.0;
      if (t < q1) {
        const bool wrap = t >= n1;
        const int jr = wrap ? b0 + (t - n1) : a0 + t;
        const bool ok = act && (wrap ? jr >= c.y : (jr >= c.x && jr < l));
        if (ok) v[u] = colpart[upb[jr] + (wrap ? (int64_t)l + M - jr : (int64_t)(l - jr))];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += v[u];
  }
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && act) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kReduceWaves; ++w) t += part[w][lane];
    out[l] = scale[l] * (rowacc[l] + t);
  }
}

__global__ void __launch_bounds__(64 * kReduceWaves)
k_local_sym_reduce(int M, const int2* __restrict__ cov, const int64_t* __restrict__ upb,
                   const double* __restrict__ rowacc, const double* __restrict__ colpart,
                   const double* __restrict__ scale, double* __restrict__ out) {
  k_local_sym_reduce_body(M, cov, upb, rowacc, colpart, scale, out, blockIdx.x);
}

// Lag 1 of the pair-once stored local sum, added to the lags >= 2 total
// `base` (already scaled): row l's own lag-1 run Q_1(d) sigma^{L-1} over the
// first c_l1 sources of its upper range, and the column terms of the rows
// j = l - k (k = 1 .. kmax, modulo M in the periodic box) whose lag-1 run
// reaches l (k < c_j1).  The runs are short (pairs closer than about p/2 dt)
// but number up to ~100 in dense media: 16 lanes per row (16 rows per
// workgroup), each lane over every 16th term, the lanes' sums added by a
// fixed butterfly.
__global__ void __launch_bounds__(256)
k_local_sym_lag1(int M, int NQ, int NH, int64_t L, int periodic, int kmax, const int64_t* __restrict__ rb,
                 const uint2* __restrict__ sacx, const double* __restrict__ Qs, const double* __restrict__ hist,
                 const double* __restrict__ scale, const double* __restrict__ base, double* __restrict__ out) {
  const int g = threadIdx.x & 15;
  const int l = blockIdx.x * 16 + (threadIdx.x >> 4);
  const bool act = l < M;   // every lane stays for the butterfly
  double a = 0.0;
  if (act) {
    const double* __restrict__ h = hist + (int64_t)mod_slot(L - 1, NH) * M;
    const uint2 c = sacx[(int64_t)l * NQ + 1];
    const double* __restrict__ q = Qs + rb[l] + c.y;
    for (int i = g; i < (int)c.x; i += 16) {
      int ll = l + i;
      if (ll >= M) ll -= M;
      a = fma(q[i], h[ll], a);
    }
    for (int k = 1 + g; k <= kmax; k += 16) {
      int j = l - k;
      if (j < 0) {
        if (!periodic) break;
        j += M;
      }
      const uint2 cj = sacx[(int64_t)j * NQ + 1];
      if (k < (int)cj.x) a = fma(Qs[rb[j] + cj.y + k], h[j], a);
    }
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
  if (act && g == 0) out[l] = base[l] + scale[l] * a;
}



// Driving data g_j(t) = beta_j f(x_j - t) (eq. (gj); f periodised in the
// periodic box), stored negated: ginc_j = -g_j.  Thread (row, packet) sums the
// packet's images; the packets are then added in order.  `pp` = packets per
// row rounded up to a power of two; 256/pp rows per block.  With deriv != 0 it
// writes f'(x_j - t) instead (gradient with respect to positions).
__device__ __forceinline__ void k_incident_body(int M, double t, const double* __restrict__ xs, const double* __restrict__ beta, Packets pk, int pp,
           int deriv, double* __restrict__ ginc, int bid) {
  __shared__ double term[256];
  const int rpb = 256 / pp;
  const int lr = threadIdx.x / pp, ip = threadIdx.x - lr * pp;
  const int j = bid * rpb + lr;
  double f = 0.0;
  if (j < M && ip < pk.n) {
    double s = xs[j] - t;
    if (pk.periodic) s -= kTwoPi * rint(s * kInvTwoPi);
    const double a = pk.p[5 * ip], c = pk.p[5 * ip + 1], wd = pk.p[5 * ip + 2];
    const double om = pk.p[5 * ip + 3], ph = pk.p[5 * ip + 4];
    const double lim = 40.0 * wd;   // exp(-y^2/(2 w^2)) underflows to 0 beyond
    const int i0 = pk.periodic ? -4 : 0, i1 = pk.periodic ? 4 : 0;
    for (int im = i0; im <= i1; ++im) {
      const double y = (s + kTwoPi * im) - c;
      if (fabs(y) < lim) {
        const double env = a * exp(-y * y / (2.0 * wd * wd));
        if (deriv) f += env * (-(y / (wd * wd)) * cos(om * y + ph) - om * sin(om * y + ph));
        else f += env * cos(om * y + ph);
      }
    }
  }
  term[threadIdx.x] = f;
  __syncthreads();
  if (ip == 0 && j < M) {
    double tot = 0.0;
    for (int q = 0; q < pk.n; ++q) tot += term[lr * pp + q];
    ginc[j] = deriv ? tot : -beta[j] * tot;
  }
}

__global__ void __launch_bounds__(256)
k_incident(int M, double t, const double* __restrict__ xs, const double* __restrict__ beta, Packets pk, int pp,
           int deriv, double* __restrict__ ginc) {
  k_incident_body(M, t, xs, beta, pk, pp, deriv, ginc, blockIdx.x);
}

// Driving data of gridDim.y consecutive levels L0, L0 + 1, ... (row y of out
// for level L0 + y): the values k_incident writes level by level.
__global__ void __launch_bounds__(256)
k_incident_levels(int M, int64_t L0, double dt, const double* __restrict__ xs, const double* __restrict__ beta,
                  Packets pk, int pp, double* __restrict__ out) {
  const int64_t L = L0 + blockIdx.y;
  k_incident_body(M, (double)L * dt, xs, beta, pk, pp, 0, out + (int64_t)blockIdx.y * M, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Per-step solve (I + S) sigma^L = rhs, S_jl = (beta_j/2) Q_0(d_jl) for d < dt
// (eq. (linearSystem)), by `iters` Jacobi sweeps from zero, one block per tile
// of consecutive rows.  The block holds the tile plus a halo of every point
// within `iters` couplings of it (rows r0..r0+el-1 of the tile matrices, with
// column indices local to that range), so the tile's result equals `iters`
// global sweeps.  The right-hand side is completed here:
//   rhs_j = part_j - beta_j u_H(x_j)
// with part_j = -g_j - (local sum) and u_H(x_j) interpolated from the type-2
// grid.  The result goes to the
// history slot of level L and, when requested, to the caller's output row.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void k_solve_body(int M, int iters, int ext_max, const int* __restrict__ tile_r0, const int* __restrict__ tile_el,
        const int* __restrict__ tile_g0, const int* __restrict__ tile_left, const int* __restrict__ tile_n,
        const int* __restrict__ rg, const double* __restrict__ rdinv, const int* __restrict__ rptr,
        const int* __restrict__ ecol, const double* __restrict__ ev, const double* __restrict__ ginc,
        const double* __restrict__ loc, const int* __restrict__ i0s, const double* __restrict__ iw,
        const double* __restrict__ beta, const double* __restrict__ grid2, int nf, int width,
        double* __restrict__ sig_out,
        double* __restrict__ save_row, const int* __restrict__ perm, int bid) {
  extern __shared__ double sm[];
  const int t = bid;
  const int r0 = tile_r0[t], el = tile_el[t];
  const int k0 = rptr[r0], ne = rptr[r0 + el] - k0;
  double* c = sm;
  double* s0 = sm + ext_max;
  double* s1 = sm + 2 * ext_max;
  double* dinv = sm + 3 * ext_max;
  double* val = sm + 4 * ext_max;                    // ne entries
  int* col = (int*)(val + ne);                       // ne entries
  int* ptr = col + ne;                               // el + 1 entries
  for (int k = threadIdx.x; k < ne; k += blockDim.x) {
    val[k] = ev[k0 + k];
    col[k] = ecol[k0 + k];
  }
  for (int e = threadIdx.x; e <= el; e += blockDim.x) ptr[e] = rptr[r0 + e] - k0;
  for (int e = threadIdx.x; e < el; e += blockDim.x) {
    const int g = rg[r0 + e];
    const double uh = interp_pre(g, i0s, iw, grid2, nf, width);
    const double cv = (ginc[g] - loc[g]) - beta[g] * uh;
    const double di = rdinv[r0 + e];
    c[e] = cv;
    dinv[e] = di;
    s0[e] = cv * di;
  }
  __syncthreads();
  for (int it = 1; it < iters; ++it) {
    for (int e = threadIdx.x; e < el; e += blockDim.x) {
      double acc = c[e];
      const int k1 = ptr[e + 1];
      for (int k = ptr[e]; k < k1; ++k) acc = fma(-val[k], s0[col[k]], acc);
      s1[e] = acc * dinv[e];
    }
    __syncthreads();
    double* tmp = s0;
    s0 = s1;
    s1 = tmp;
  }
  const int g0 = tile_g0[t], left = tile_left[t], nt = tile_n[t];
  for (int k = threadIdx.x; k < nt; k += blockDim.x) {
    int g = g0 + k;
    if (g >= M) g -= M;   // a run may wrap around the periodic box
    const double v = s0[left + k];
    sig_out[g] = v;
    if (save_row) save_row[perm[g]] = v;
  }
}

__global__ void __launch_bounds__(256)
k_solve(int M, int iters, int ext_max, const int* __restrict__ tile_r0, const int* __restrict__ tile_el,
        const int* __restrict__ tile_g0, const int* __restrict__ tile_left, const int* __restrict__ tile_n,
        const int* __restrict__ rg, const double* __restrict__ rdinv, const int* __restrict__ rptr,
        const int* __restrict__ ecol, const double* __restrict__ ev, const double* __restrict__ ginc,
        const double* __restrict__ loc, const int* __restrict__ i0s, const double* __restrict__ iw,
        const double* __restrict__ beta, const double* __restrict__ grid2, int nf, int width,
        double* __restrict__ sig_out,
        double* __restrict__ save_row, const int* __restrict__ perm) {
  k_solve_body(M, iters, ext_max, tile_r0, tile_el, tile_g0, tile_left, tile_n, rg, rdinv, rptr, ecol, ev, ginc, loc, i0s, iw, beta, grid2, nf, width, sig_out, save_row, perm, blockIdx.x);
}

// Per-step solve when the tiles do not fit in LDS (dense nearby coupling along
// long runs): global Jacobi sweeps, one launch each, CSR over all rows.
// k_solve_rhs completes the right-hand side b_j = part_j - beta_j u_H(x_j) and
// the first sweep from zero, x_j = b_j / (1 + S_jj); k_jacobi_sweep does
// x'_j = (b_j - sum_{l != j} S_jl x_l) / (1 + S_jj) and, on the last sweep,
// also writes the caller's row.
__device__ __forceinline__ void k_solve_rhs_body(int M, const double* __restrict__ ginc, const double* __restrict__ loc,
                            const double* __restrict__ beta, const int* __restrict__ i0s,
                            const double* __restrict__ iw, const double* __restrict__ grid2, int nf, int width,
                            const double* __restrict__ dinv, double* __restrict__ rhs, double* __restrict__ x, int bid) {
  const int j = bid * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const double b = (ginc[j] - loc[j]) - beta[j] * interp_pre(j, i0s, iw, grid2, nf, width);
  rhs[j] = b;
  x[j] = b * dinv[j];
}

__global__ void k_solve_rhs(int M, const double* __restrict__ ginc, const double* __restrict__ loc,
                            const double* __restrict__ beta, const int* __restrict__ i0s,
                            const double* __restrict__ iw, const double* __restrict__ grid2, int nf, int width,
                            const double* __restrict__ dinv, double* __restrict__ rhs, double* __restrict__ x) {
  k_solve_rhs_body(M, ginc, loc, beta, i0s, iw, grid2, nf, width, dinv, rhs, x, blockIdx.x);
}

__device__ __forceinline__ void k_jacobi_sweep_body(int M, const int* __restrict__ ptr, const int* __restrict__ col,
                               const double* __restrict__ val, const double* __restrict__ dinv,
                               const double* __restrict__ rhs, const double* __restrict__ xin,
                               double* __restrict__ xout, double* __restrict__ save_row,
                               const int* __restrict__ perm, int bid) {
  const int j = bid * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double acc = rhs[j];
  for (int k = ptr[j]; k < ptr[j + 1]; ++k) acc = fma(-val[k], xin[col[k]], acc);
  const double v = acc * dinv[j];
  xout[j] = v;
  if (save_row) save_row[perm[j]] = v;
}

__global__ void k_jacobi_sweep(int M, const int* __restrict__ ptr, const int* __restrict__ col,
                               const double* __restrict__ val, const double* __restrict__ dinv,
                               const double* __restrict__ rhs, const double* __restrict__ xin,
                               double* __restrict__ xout, double* __restrict__ save_row,
                               const int* __restrict__ perm) {
  k_jacobi_sweep_body(M, ptr, col, val, dinv, rhs, xin, xout, save_row, perm, blockIdx.x);
}

// The same sweep with one wavefront per row (lanes over the row's entries),
// for rows with many nearby sources: the entry loads coalesce.
__device__ __forceinline__ void k_jacobi_sweep_wave_body(int M, const int* __restrict__ ptr,
                               const int* __restrict__ col, const double* __restrict__ val,
                               const double* __restrict__ dinv, const double* __restrict__ rhs,
                               const double* __restrict__ xin, double* __restrict__ xout,
                               double* __restrict__ save_row, const int* __restrict__ perm, int bid) {
  const int lane = threadIdx.x & 63;
  const int j = bid * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= M) return;
  double acc = 0.0;
  for (int k = ptr[j] + lane; k < ptr[j + 1]; k += 64) acc = fma(val[k], xin[col[k]], acc);
  acc = wave_sum(acc);
  if (lane == 0) {
    const double v = (rhs[j] - acc) * dinv[j];
    xout[j] = v;
    if (save_row) save_row[perm[j]] = v;
  }
}

__global__ void __launch_bounds__(256)
k_jacobi_sweep_wave(int M, const int* __restrict__ ptr, const int* __restrict__ col,
                    const double* __restrict__ val, const double* __restrict__ dinv,
                    const double* __restrict__ rhs, const double* __restrict__ xin, double* __restrict__ xout,
                    double* __restrict__ save_row, const int* __restrict__ perm) {
  k_jacobi_sweep_wave_body(M, ptr, col, val, dinv, rhs, xin, xout, save_row, perm, blockIdx.x);
}

// Per-step solve on small nearby-runs: I + S is block diagonal over maximal
// runs of consecutive springs closer than dt; a run of s springs is solved with
// its precomputed inverse,  sigma_i = sum_k inv[i][k] rhs_k.  One block per
// tile of whole runs (points g0 .. g0 + n - 1, circular).  Per point: the
// run's first local index, its size and the offset of its inverse row.
__device__ __forceinline__ void k_solve_direct_body(int M, const int* __restrict__ dt_g0, const int* __restrict__ dt_n, const int* __restrict__ dt_p0,
               const int* __restrict__ pt_cs, const int* __restrict__ pt_cn, const int64_t* __restrict__ pt_inv,
               const double* __restrict__ inv, const double* __restrict__ ginc, const double* __restrict__ loc,
               const int* __restrict__ i0s, const double* __restrict__ iw, const double* __restrict__ beta,
               const double* __restrict__ grid2, int nf, int width, double* __restrict__ sig_out,
               double* __restrict__ save_row, const int* __restrict__ perm, int bid) {
  __shared__ double c[256];
  const int t = bid;
  const int g0 = dt_g0[t], n = dt_n[t], p0 = dt_p0[t];
  const int e = threadIdx.x;
  int g = g0 + e;
  if (g >= M) g -= M;
  if (e < n) c[e] = (ginc[g] - loc[g]) - beta[g] * interp_pre(g, i0s, iw, grid2, nf, width);
  __syncthreads();
  if (e < n) {
    const int cs = pt_cs[p0 + e], cn = pt_cn[p0 + e];
    const double* __restrict__ row = inv + pt_inv[p0 + e];
    double acc = 0.0;
    for (int k = 0; k < cn; ++k) acc = fma(row[k], c[cs + k], acc);
    sig_out[g] = acc;
    if (save_row) save_row[perm[g]] = acc;
  }
}

__global__ void __launch_bounds__(256)
k_solve_direct(int M, const int* __restrict__ dt_g0, const int* __restrict__ dt_n, const int* __restrict__ dt_p0,
               const int* __restrict__ pt_cs, const int* __restrict__ pt_cn, const int64_t* __restrict__ pt_inv,
               const double* __restrict__ inv, const double* __restrict__ ginc, const double* __restrict__ loc,
               const int* __restrict__ i0s, const double* __restrict__ iw, const double* __restrict__ beta,
               const double* __restrict__ grid2, int nf, int width, double* __restrict__ sig_out,
               double* __restrict__ save_row, const int* __restrict__ perm) {
  k_solve_direct_body(M, dt_g0, dt_n, dt_p0, pt_cs, pt_cn, pt_inv, inv, ginc, loc, i0s, iw, beta, grid2, nf, width, sig_out, save_row, perm, blockIdx.x);
}

// Field at the receivers, one wavefront per receiver:
//   u(x_r, t_L) = sum_{m>=0} sum_l (1/2) Q_m(d_rl) sigma_l^{L-m} + u_H(x_r)
__device__ __forceinline__ void k_receivers_body(int R, int M, int NQ, int NH, int64_t L,
            const int* __restrict__ nb_start, const int* __restrict__ nb_count, const int64_t* __restrict__ qoff,
            const double* __restrict__ Q, const double* __restrict__ hist, const int* __restrict__ i0s,
            const double* __restrict__ iw, const double* __restrict__ grid2, int nf, int width,
            double* __restrict__ out, int bid) {
  const int lane = threadIdx.x & 63;
  const int r = bid * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= R) return;   // no block-level barrier in this body
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
  if (lane == 0) out[r] = acc + interp_pre(r, i0s, iw, grid2, nf, width);
}

// The same with a workgroup of 16 wavefronts per receiver (receivers are few
// and may have thousands of neighbours, so one wavefront each leaves most of
// the chip idle and waits on one load at a time): wavefront w takes the lags
// m = w, w + 16, ..., its lanes the sources, four loads in flight per lane;
// the wavefronts' sums are added in a fixed order.
__global__ void __launch_bounds__(1024)
k_receivers(int M, int NQ, int NH, int64_t L, const int* __restrict__ nb_start, const int* __restrict__ nb_count,
            const int64_t* __restrict__ qoff, const double* __restrict__ Q, const double* __restrict__ hist,
            const int* __restrict__ i0s, const double* __restrict__ iw, const double* __restrict__ grid2, int nf,
            int width, double* __restrict__ out) {
  __shared__ double part[16];
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = nb_count[r], st = nb_start[r];
  const int64_t base = qoff[r];
  double acc = 0.0;
  for (int m = wv; m < NQ; m += 16) {
    const double* __restrict__ sl = hist + (int64_t)mod_slot(L - m, NH) * M;
    const double* __restrict__ qm = Q + base + (int64_t)m * n;
    for (int i0 = 0; i0 < n; i0 += 256) {
      double q[4], h[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + lane + 64 * u;
        q[u] = 0.0;
        h[u] = 0.0;
        if (i < n) {
          int l = st + i;
          if (l >= M) l -= M;
          q[u] = qm[i];
          h[u] = sl[l];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = fma(q[u], h[u], acc);
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) part[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < 16; ++w) sum += part[w];
    out[r] = sum + interp_pre(r, i0s, iw, grid2, nf, width);
  }
}

// Element k of the packed input of the u (or v) grid transform from the modes
// a: z_k = conj of (y_k + conj y_{K-k}) + i e^{+i pi k/K} (y_k - conj y_{K-k}),
// y_k = (-1)^k conj(a_k); tw[k] = e^{-i pi k/K}.
__device__ __forceinline__ double2 rbc_grid_in(int64_t k, int64_t K, int n1, int n2, const double2* __restrict__ a,
                                               const double2* __restrict__ tw) {
  const double sk = (k & 1) ? -1.0 : 1.0;
  const double2 yk = cscale(cconj(a[mode_pos(k, n1, n2)]), sk);
  double2 ym = make_double2(0.0, 0.0);
  if (k > 0) {
    const int64_t km = K - k;
    const double sm = (km & 1) ? -1.0 : 1.0;
    ym = cconj(cscale(cconj(a[mode_pos(km, n1, n2)]), sm));
  }
  return cconj(cadd(cadd(yk, ym), cmul_pi(cmul(cconj(tw[k]), csub(yk, ym)))));
}

// Grid values 2j and 2j+1 of u (is_v = false) or v after the roll-off on
// |i - K| >= K - 2W, packed as one complex input of the transform back.
__device__ __forceinline__ double2 rbc_modes_in(int64_t j, int64_t K, int W, double h, double delta_s, bool is_v,
                                                const double* __restrict__ cheb_phi, const double* __restrict__ cheb_g,
                                                int ncheb, const double* __restrict__ gu,
                                                const double* __restrict__ gv) {
  double val[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int64_t ip = 2 * j + e;       // grid index 0..2K-1
    const int64_t i = ip - K;           // -K..K-1
    const int64_t ai = i < 0 ? -i : i;
    double u = gu[ip];
    double v = is_v ? gv[ip] : 0.0;
    if (ai >= K - 2 * W) {
      const double arg = (double)(K - ai - W) * h;
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
  return make_double2(val[0], val[1]);
}

// Mode k (< K) from the transform Z of the rolled-off grid (real transform of
// length 2K unpacked): alpha_k = (1/2K) (-1)^k conj(X_k).
__device__ __forceinline__ double2 rbc_modes_out(int64_t k, int64_t K, const double2* __restrict__ Z,
                                                 const double2* __restrict__ tw) {
  const double2 zk = Z[k];
  const double2 zc = cconj(Z[k == 0 ? 0 : K - k]);
  const double2 E = cscale(cadd(zk, zc), 0.5);
  const double2 O = cscale(cmul_mi(csub(zk, zc)), 0.5);
  const double2 X = cadd(E, cmul(tw[k], O));
  const double sk = (k & 1) ? -1.0 : 1.0;
  return cscale(cconj(X), sk * (1.0 / (2.0 * (double)K)));
}

// ---------------------------------------------------------------------------
// Free-space RBC projection (Section 4.4).  Block 0 handles alpha -> u,
// block 1 alpha' -> v: values on x_i = -pi + i h, i = 0..2K-1 (h = pi/K), from
// the modes |k| < K (k = K dropped): grid = c2r of y_k = (-1)^k conj(a_k).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
k_rbc_to_grid(FftPlan fp, int64_t K, int n1, int n2, const double2* __restrict__ alpha,
              const double2* __restrict__ dalpha, const double2* __restrict__ tw, double2* __restrict__ gu,
              double2* __restrict__ gv) {
  extern __shared__ double2 buf[];
  const double2* __restrict__ a = (blockIdx.x == 0) ? alpha : dalpha;
  double2* __restrict__ out = (blockIdx.x == 0) ? gu : gv;
  const int n = fp.n;  // == K
  for (int k = threadIdx.x; k < n; k += blockDim.x) buf[k] = rbc_grid_in(k, K, n1, n2, a, tw);
  __syncthreads();
  fft_lds(buf, fp, tw, 2);
  for (int j = threadIdx.x; j < n; j += blockDim.x) out[j] = cconj(buf[j]);
}

// Roll-off on |i - K| >= K - 2W with the spatial window (delta_s = W h):
//   u~ = phi_s(a) u,  v~ = phi_s'(a) u + phi_s(a) v,  a = (K - |i - K| - W) h,
// then back to modes alpha_k = (1/2K) (-1)^k conj(X_k), k < K, alpha_K = 0.
// Block 0 writes alpha and the type-2 input y, block 1 writes alpha'.
__global__ void __launch_bounds__(1024)
k_rbc_to_modes(FftPlan fp, int64_t K, int n1, int n2, int W, double h, double delta_s,
               const double* __restrict__ cheb_phi,
               const double* __restrict__ cheb_g, int ncheb, const double* __restrict__ gu,
               const double* __restrict__ gv, const double2* __restrict__ tw, const double* __restrict__ dk2,
               double2* __restrict__ alpha, double2* __restrict__ dalpha, double2* __restrict__ y) {
  extern __shared__ double2 buf[];
  const int n = fp.n;       // == K complex, 2K real points
  const bool is_v = blockIdx.x == 1;
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    buf[j] = rbc_modes_in(j, K, W, h, delta_s, is_v, cheb_phi, cheb_g, ncheb, gu, gv);
  __syncthreads();
  fft_lds(buf, fp, tw, 2);
  // unpack the real transform of length 2K and return to modes
  double2* __restrict__ out = is_v ? dalpha : alpha;
  for (int k = threadIdx.x; k <= n; k += blockDim.x) {
    const double2 a = k < n ? rbc_modes_out(k, K, buf, tw) : make_double2(0.0, 0.0);
    const int64_t pos = mode_pos(k, n1, n2);
    out[pos] = a;
    if (!is_v) y[k] = cscale(cconj(a), dk2[pos]);
  }
}


// ---------------------------------------------------------------------------
// The same projection for grids too long for one workgroup (K complex points,
// K = a b): the length-K transform runs in four steps over workgroups,
//   pass 1, block (j1, s): FFT over j2 of z_s[j1 + a j2], j2 < b, times
//           e^{-2 pi i j1 k2 / K} -> T_s[k2 a + j1];
//   pass 2, block (k2, s): FFT over j1 of T_s[k2 a + j1], j1 < a
//           -> X_s[k2 + b k1],
// with s = 0 for u (from alpha) and s = 1 for v (from alpha'), each sequence
// K long.  The packing before and the unpacking after the transform are the
// elementwise steps of the one-workgroup kernels above.  tw[t] = e^{-2 pi i t / (2K)}.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_rbc_grid_pack(int64_t K, int n1, int n2, const double2* __restrict__ alpha, const double2* __restrict__ dalpha,
                const double2* __restrict__ tw, double2* __restrict__ z) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * K) return;
  const int sidx = idx >= K ? 1 : 0;
  z[idx] = rbc_grid_in(idx - sidx * K, K, n1, n2, sidx ? dalpha : alpha, tw);
}

__global__ void __launch_bounds__(256)
k_rbc_fft_pass1(FftPlan fb, int a, int64_t K, const double2* __restrict__ tw, const double2* __restrict__ z,
                double2* __restrict__ T) {
  extern __shared__ double2 buf[];
  const int b = fb.n, j1 = blockIdx.x;
  const int64_t off = (int64_t)blockIdx.y * K;
  for (int j2 = threadIdx.x; j2 < b; j2 += blockDim.x) buf[j2] = z[off + j1 + (int64_t)a * j2];
  __syncthreads();
  fft_batch(buf, 1, fb, tw, 2 * a);
  for (int k2 = threadIdx.x; k2 < b; k2 += blockDim.x)
    T[off + (int64_t)k2 * a + j1] = cmul(buf[k2], tw[2 * (int64_t)j1 * k2]);   // j1 k2 < K
}

__global__ void __launch_bounds__(256)
k_rbc_fft_pass2(FftPlan fa, int b, int64_t K, const double2* __restrict__ tw, const double2* __restrict__ T,
                double2* __restrict__ out0, double2* __restrict__ out1, int conj_out) {
  extern __shared__ double2 buf[];
  const int a = fa.n, k2 = blockIdx.x;
  const int64_t off = (int64_t)blockIdx.y * K;
  double2* __restrict__ out = blockIdx.y ? out1 : out0;
  for (int j1 = threadIdx.x; j1 < a; j1 += blockDim.x) buf[j1] = T[off + (int64_t)k2 * a + j1];
  __syncthreads();
  fft_batch(buf, 1, fa, tw, 2 * b);
  for (int k1 = threadIdx.x; k1 < a; k1 += blockDim.x) {
    const double2 v = buf[k1];
    out[k2 + (int64_t)b * k1] = conj_out ? cconj(v) : v;
  }
}

__global__ void __launch_bounds__(256)
k_rbc_modes_pack(int64_t K, int W, double h, double delta_s, const double* __restrict__ cheb_phi,
                 const double* __restrict__ cheb_g, int ncheb, const double* __restrict__ gu,
                 const double* __restrict__ gv, double2* __restrict__ z) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * K) return;
  const bool is_v = idx >= K;
  z[idx] = rbc_modes_in(idx - (is_v ? K : 0), K, W, h, delta_s, is_v, cheb_phi, cheb_g, ncheb, gu, gv);
}

__global__ void __launch_bounds__(256)
k_rbc_modes_unpack(int64_t K, int n1, int n2, const double2* __restrict__ X, const double2* __restrict__ tw,
                   const double* __restrict__ dk2, double2* __restrict__ alpha, double2* __restrict__ dalpha,
                   double2* __restrict__ y) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * (K + 1)) return;
  const bool is_v = idx > K;
  const int64_t k = idx - (is_v ? K + 1 : 0);
  const double2 a = k < K ? rbc_modes_out(k, K, X + (is_v ? K : 0), tw) : make_double2(0.0, 0.0);
  const int64_t pos = mode_pos(k, n1, n2);
  (is_v ? dalpha : alpha)[pos] = a;
  if (!is_v) y[k] = cscale(cconj(a), dk2[pos]);
}

// ===========================================================================
// History part of one level as three kernels.  The half-length complex
// transform of the fine grid (n = N/2 points, N = n_f) is done in four steps
// with n = n1 n2:  j = j1 + n1 j2,  k = k2 + n2 k1,
//   X_{k2 + n2 k1} = sum_j1 w_n1^{j1 k1} [ w_n^{j1 k2} sum_j2 z_{j1 + n1 j2} w_n2^{j2 k2} ].
// A: for one j1, spread the 2 n2 grid cells of z_{j1 + n1 j2}, FFT over j2,
//    twiddle, store T1[k2][j1].
// B: for the column pair {k2, n2 - k2} (which holds both k and n - k, as the
//    real-transform unpacking needs): FFT over j1 -> X_k; spectra, FIR and
//    propagator for the k <= K in these columns; pack the type-2 spectrum and
//    run the first inverse step (FFT over k1, twiddle) -> V[j1][k2].
// C: for one j1, inverse FFT over k2 -> z_{j1 + n1 j2} -> grid cells.
// ===========================================================================
__device__ __forceinline__ double spread_cell(int cell, const double* __restrict__ sig, int M,
                                              const int* __restrict__ cstart, const int* __restrict__ ccount,
                                              const int64_t* __restrict__ woff, const double* __restrict__ sw) {
  const int st = cstart[cell], cnt = ccount[cell];
  const double* __restrict__ w = sw + woff[cell];
  double acc = 0.0;
  for (int c = 0; c < cnt; ++c) {
    int j = st + c;
    if (j >= M) j -= M;
    acc = fma(sig[j], w[c], acc);
  }
  return acc;
}

__device__ __forceinline__ void k_hist_a_body(FftPlan f2, int n1, const double* __restrict__ sig, int M, const int* __restrict__ cstart,
         const int* __restrict__ ccount, const int64_t* __restrict__ woff, const double* __restrict__ sw,
         const double2* __restrict__ tw, double2* __restrict__ T1, ExtraSources ex, int bid,
         const double* __restrict__ grid = nullptr) {
  extern __shared__ double2 buf[];
  const int n2 = f2.n, j1 = bid;
  const int n = n1 * n2;
  double* bd = (double*)buf;
  for (int c = threadIdx.x; c < 2 * n2; c += blockDim.x) {
    const int cell = 2 * (j1 + n1 * (c >> 1)) + (c & 1);
    if (grid) {
      bd[c] = grid[cell];   // spread beforehand by k_spread_grid
      continue;
    }
    double v = spread_cell(cell, sig, M, cstart, ccount, woff, sw);
    if (ex.val) v += spread_cell(cell, ex.val, ex.n, ex.cstart, ex.ccount, ex.woff, ex.w);
    bd[c] = v;
  }
  __syncthreads();
  fft_batch(buf, 1, f2, tw, 2 * n1);
  for (int k2 = threadIdx.x; k2 < n2; k2 += blockDim.x) {
    const int q = j1 * k2;                 // < n
    T1[(int64_t)k2 * n1 + j1] = cmul(buf[k2], tw[2 * (q % n)]);
  }
}

__global__ void __launch_bounds__(256)
k_hist_a(FftPlan f2, int n1, const double* __restrict__ sig, int M, const int* __restrict__ cstart,
         const int* __restrict__ ccount, const int64_t* __restrict__ woff, const double* __restrict__ sw,
         const double2* __restrict__ tw, double2* __restrict__ T1, ExtraSources ex) {
  k_hist_a_body(f2, n1, sig, M, cstart, ccount, woff, sw, tw, T1, ex, blockIdx.x);
}

// Rows longer than 1024 butterflies per stage for 256 threads take 1024 threads.
// Long rows: the cells are spread beforehand into `grid` by k_spread_grid (one
// thread per cell, coalesced), and the rows are read from it; blocks of
// neighbouring rows share the grid's cache lines, so they run on one XCD.  The
// grid is padded to a multiple of 8 blocks (the remap's bijection); blocks
// past the last row return as a whole, before any barrier.
__global__ void __launch_bounds__(1024)
k_hist_a_wide(FftPlan f2, int n1, const double* __restrict__ grid, const double2* __restrict__ tw,
              double2* __restrict__ T1) {
  const int j1 = xcd_block(blockIdx.x, gridDim.x);
  if (j1 >= n1) return;
  const ExtraSources none{nullptr, 0, nullptr, nullptr, nullptr, nullptr};
  k_hist_a_body(f2, n1, nullptr, 0, nullptr, nullptr, nullptr, nullptr, tw, T1, none, j1, grid);
}

// Type-1 spreading onto the fine grid, one thread per cell.
__global__ void __launch_bounds__(256)
k_spread_grid(int nf, const double* __restrict__ sig, int M, const int* __restrict__ cstart,
              const int* __restrict__ ccount, const int64_t* __restrict__ woff, const double* __restrict__ sw,
              ExtraSources ex, double* __restrict__ grid) {
  const int cell = blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= nf) return;
  double v = spread_cell(cell, sig, M, cstart, ccount, woff, sw);
  if (ex.val) v += spread_cell(cell, ex.val, ex.n, ex.cstart, ex.ccount, ex.woff, ex.w);
  grid[cell] = v;
}

constexpr int kFirGroups = 8;

// Partner of position (c, k1) in the column pair: where Z_{n - q} sits, q = col[c] + n2 k1.
__device__ __forceinline__ int partner(int c, int k1, int k2c, int ncol, int n1) {
  if (k2c == 0) return c * n1 + (n1 - k1) % n1;
  const int cp = (ncol == 2) ? 1 - c : c;
  return cp * n1 + (n1 - 1 - k1);
}

// mode 0: forward step 2 + modes + inverse step 1; mode 1: forward step 2 +
// modes, writing y (the type-2 input) for a later projection; mode 2: inverse
// step 1 from y.
__device__ __forceinline__ void k_hist_b_body(int mode, FftPlan f1, int n2, int64_t K, int W, int64_t L, int64_t npos, const double2* __restrict__ T1,
         const double2* __restrict__ tw, const double2* __restrict__ tw1, const double* __restrict__ dk1, const double* __restrict__ dk2,
         const double* __restrict__ pk, const double* __restrict__ qk, const double* __restrict__ rot,
         double2* __restrict__ ring, double2* __restrict__ alpha, double2* __restrict__ dalpha,
         double2* __restrict__ y, double2* __restrict__ V, int G, int bid, int vcol = 0) {
  extern __shared__ double2 smb[];
  const int n1 = f1.n;
  const int n = n1 * n2;
  double2* buf = smb;                         // [2][n1]
  double2* yl = smb + 2 * n1;                 // [2][n1]
  double2* sS = smb + 4 * n1;                 // [2][n1]
  double4* red = (double4*)(smb + 6 * n1);    // [G][2 n1]
  const int k2a = bid, k2b = (n2 - k2a) % n2;
  const int ncol = (k2a == k2b) ? 1 : 2;
  const int np = ncol * n1;
  const int64_t stride = npos;
  const int64_t pb = (int64_t)k2a * 2 * n1;   // position of this block's first mode
  auto colk2 = [&](int c) { return c == 0 ? k2a : k2b; };
  if (mode != 2) {
    for (int e = threadIdx.x; e < np; e += blockDim.x) {
      const int c = e / n1, k1 = e - c * n1;
      buf[e] = T1[(int64_t)colk2(c) * n1 + k1];
    }
    __syncthreads();
    fft_batch(buf, ncol, f1, tw, 2 * n2);
    const int64_t nn = L - 1;
    // spectra S_q of the modes q <= K held by this block
    for (int e = threadIdx.x; e < np; e += blockDim.x) {
      const int c = e / n1, k1 = e - c * n1;
      const int64_t q = colk2(c) + (int64_t)n2 * k1;
      double2 S = make_double2(0.0, 0.0);
      if (q <= K) {
        const double2 zk = buf[e];
        const double2 zc = cconj(buf[partner(c, k1, k2a, ncol, n1)]);
        const double2 E = cscale(cadd(zk, zc), 0.5);
        const double2 O = cscale(cmul_mi(csub(zk, zc)), 0.5);
        // e^{-2 pi i q / N} = e^{-2 pi i k2 / N} e^{-2 pi i k1 / (2 n1)}: the column's
        // factor and a short table instead of a stride-n2 gather
        const double2 X = cadd(E, cmul(cmul(tw[colk2(c)], tw1[k1]), O));
        S = cscale(cconj(X), dk1[pb + e]);
      }
      sS[e] = S;
    }
    __syncthreads();
    // FIR partial sums: work item (e, g) takes taps m = g, g + G, ...
    for (int wi = threadIdx.x; wi < np * G; wi += blockDim.x) {
      const int g = wi / np, e = wi - g * np;
      const int c = e / n1, k1 = e - c * n1;
      const int64_t q = colk2(c) + (int64_t)n2 * k1;
      double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
      if (q <= K) {
#pragma unroll 2
        for (int m = g; m < W; m += G) {
          const double2 Sm = (m == 0) ? sS[e] : ring[(int64_t)mod_slot(nn - m, W) * stride + pb + e];
          const double p = pk[(int64_t)m * stride + pb + e], qq = qk[(int64_t)m * stride + pb + e];
          acc.x = fma(p, Sm.x, acc.x);
          acc.y = fma(p, Sm.y, acc.y);
          acc.z = fma(qq, Sm.x, acc.z);
          acc.w = fma(qq, Sm.y, acc.w);
        }
      }
      red[g * np + e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < np; e += blockDim.x) {
      const int c = e / n1, k1 = e - c * n1;
      const int64_t q = colk2(c) + (int64_t)n2 * k1;
      double2 yq = make_double2(0.0, 0.0);
      if (q <= K) {
        double2 h = make_double2(0.0, 0.0), g = make_double2(0.0, 0.0);
        for (int gg = 0; gg < G; ++gg) {
          const double4 v = red[gg * np + e];
          h.x += v.x;
          h.y += v.y;
          g.x += v.z;
          g.y += v.w;
        }
        const int64_t ps = pb + e;
        ring[(int64_t)mod_slot(nn, W) * stride + ps] = sS[e];
        const double cr = rot[3 * ps], sr = rot[3 * ps + 1], rr = rot[3 * ps + 2];
        const double2 a = alpha[ps], da = dalpha[ps];
        const double2 an = make_double2(cr * a.x + sr * da.x + h.x, cr * a.y + sr * da.y + h.y);
        const double2 dan = make_double2(rr * a.x + cr * da.x + g.x, rr * a.y + cr * da.y + g.y);
        alpha[ps] = an;
        dalpha[ps] = dan;
        yq = cscale(cconj(an), dk2[ps]);
        if (mode == 1) y[q] = yq;
      }
      yl[e] = yq;
    }
    if (mode == 1) return;   // block-uniform
  } else {
    for (int e = threadIdx.x; e < np; e += blockDim.x) {
      const int c = e / n1, k1 = e - c * n1;
      const int64_t q = colk2(c) + (int64_t)n2 * k1;
      yl[e] = (q <= K) ? y[q] : make_double2(0.0, 0.0);
    }
  }
  __syncthreads();
  // pack: Z'_q = (y_q + conj(y_{n-q})) + i e^{+2 pi i q/N} (y_q - conj(y_{n-q})); buf = conj(Z')
  for (int e = threadIdx.x; e < np; e += blockDim.x) {
    const int c = e / n1, k1 = e - c * n1;
    const int q = colk2(c) + n2 * k1;
    const double2 yk = yl[e];
    const double2 ym = (q == 0) ? make_double2(0.0, 0.0) : cconj(yl[partner(c, k1, k2a, ncol, n1)]);
    const double2 zq = cadd(cadd(yk, ym), cmul_pi(cmul(cconj(cmul(tw[colk2(c)], tw1[k1])), csub(yk, ym))));
    buf[e] = cconj(zq);
  }
  __syncthreads();
  fft_batch(buf, ncol, f1, tw, 2 * n2);
  // V[j1][k2] = conj(buf) * e^{+2 pi i j1 k2 / n}
  for (int e = threadIdx.x; e < np; e += blockDim.x) {
    const int c = e / n1, j1 = e - c * n1;
    const int k2 = colk2(c);
    const int qq = (j1 * k2) % n;
    const double2 v = cmul(cconj(buf[e]), cconj(tw[2 * qq]));
    if (vcol) V[(int64_t)k2 * n1 + j1] = v;   // column-major: this column contiguous
    else V[(int64_t)j1 * n2 + k2] = v;
  }
}

// at most 128 VGPRs, so that two blocks share a compute unit: the chain runs
// its n2/2 + 1 blocks on one XCD's 32 compute units in one round
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_hist_b(int mode, FftPlan f1, int n2, int64_t K, int W, int64_t L, int64_t npos, const double2* __restrict__ T1,
         const double2* __restrict__ tw, const double2* __restrict__ tw1, const double* __restrict__ dk1,
         const double* __restrict__ dk2, const double* __restrict__ pk, const double* __restrict__ qk,
         const double* __restrict__ rot, double2* __restrict__ ring, double2* __restrict__ alpha,
         double2* __restrict__ dalpha, double2* __restrict__ y, double2* __restrict__ V, int G, int vcol) {
  k_hist_b_body(mode, f1, n2, K, W, L, npos, T1, tw, tw1, dk1, dk2, pk, qk, rot, ring, alpha, dalpha, y, V, G,
                blockIdx.x, vcol);
}

__device__ __forceinline__ void k_hist_c_body(FftPlan f2, int n1, const double2* __restrict__ V, const double2* __restrict__ tw,
         double2* __restrict__ grid2, int bid, int vcol = 0) {
  extern __shared__ double2 buf[];
  const int n2 = f2.n, j1 = bid;
  for (int k2 = threadIdx.x; k2 < n2; k2 += blockDim.x)
    buf[k2] = cconj(vcol ? V[(int64_t)k2 * n1 + j1] : V[(int64_t)j1 * n2 + k2]);
  __syncthreads();
  fft_batch(buf, 1, f2, tw, 2 * n1);
  for (int j2 = threadIdx.x; j2 < n2; j2 += blockDim.x) grid2[j1 + n1 * j2] = cconj(buf[j2]);
}

__global__ void __launch_bounds__(256)
k_hist_c(FftPlan f2, int n1, const double2* __restrict__ V, const double2* __restrict__ tw,
         double2* __restrict__ grid2) {
  k_hist_c_body(f2, n1, V, tw, grid2, blockIdx.x);
}

__global__ void __launch_bounds__(1024)
k_hist_c_wide(FftPlan f2, int n1, const double2* __restrict__ V, const double2* __restrict__ tw,
              double2* __restrict__ grid2) {
  // V column-major (written a column at a time by the column pass); neighbouring
  // rows on one XCD share its cache lines; the grid is padded to a multiple of
  // 8 blocks and blocks past the last row return as a whole
  const int j1 = xcd_block(blockIdx.x, gridDim.x);
  if (j1 >= n1) return;
  k_hist_c_body(f2, n1, V, tw, grid2, j1, 1);
}

// ---------------------------------------------------------------------------
// Gradient pass.  The transpose of one level is the same level run backwards
// in time with the adjoint densities q (solved with the same I + S) and the
// receivers acting as sources of strength dJ/du_r; see the plan for the
// bookkeeping.  These kernels are the pieces the forward level lacks.
// ---------------------------------------------------------------------------

// Type-2 input of d/dx u_H: the modes -i k alpha_k, deconvolved like y.
__global__ void k_deriv_y(int64_t K, int n1, int n2, const double2* __restrict__ alpha,
                          const double* __restrict__ dk2, double2* __restrict__ y) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q > K) return;
  const int64_t pos = mode_pos(q, n1, n2);
  // conj(-i q alpha) = i q conj(alpha)
  y[q] = cscale(cmul_pi(cconj(alpha[pos])), (double)q * dk2[pos]);
}

// Adjoint driving data of scatterer j at forward level L from the receivers
// within delta:  ginc_j = -beta_j sum_r sum_{m>=0, L+m<N} (1/2) Q_m(d_rj) e_r^{L+m}
// and (when xw is given) the position-derivative sum with the signed weights
// dQr.  e is the caller's [N][R] array dJ/du (receiver index order).
__global__ void k_adj_drive(int M, int R, int NQ, int64_t L, int64_t N, const int* __restrict__ ptr,
                            const int* __restrict__ rr, const int* __restrict__ ri,
                            const int64_t* __restrict__ rqoff, const int* __restrict__ rcount,
                            const double* __restrict__ Qr, const double* __restrict__ dQr,
                            const double* __restrict__ e, const double* __restrict__ beta,
                            double* __restrict__ ginc, double* __restrict__ xw) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  double acc = 0.0, accd = 0.0;
  for (int t = ptr[j]; t < ptr[j + 1]; ++t) {
    const int r = rr[t];
    const int n = rcount[r];
    const int64_t base = rqoff[r] + ri[t];
    for (int m = 0; m < NQ && L + m < N; ++m) {
      const double ev = e[(L + m) * R + r];
      acc = fma(Qr[base + (int64_t)m * n], ev, acc);
      if (xw) accd = fma(dQr[base + (int64_t)m * n], ev, accd);
    }
  }
  ginc[j] = -beta[j] * acc;
  if (xw) xw[j] = accd;
}

// Forward derivative data of one level: D_j = f'(x_j - t) + (signed
// derivative local sum of lags m >= 0) + d/dx u_H(x_j).
__global__ void k_fwd_dterm(int M, const double* __restrict__ fprime, const int* __restrict__ i0s,
                            const double* __restrict__ iw, const double* __restrict__ gridd, int nf, int width,
                            double* __restrict__ D) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  D[j] = fprime[j] + interp_pre(j, i0s, iw, gridd, nf, width);
}

// Accumulate one level of the gradient (sorted order):
//   gbeta_j += -q_j sigma_j / beta_j^2
//   gx_j    += q_j (D_j + Dloc_j) + sigma_j (xloc_j + xw_j + d/dx u_H^adj(x_j))
// with D = f' + d/dx u_H of the forward state and Dloc the forward
// derivative local sum.
__global__ void k_adj_grad(int M, const double* __restrict__ q, const double* __restrict__ sig,
                           const double* __restrict__ beta, const double* __restrict__ D,
                           const double* __restrict__ Dloc, const double* __restrict__ xloc,
                           const double* __restrict__ xw, const int* __restrict__ i0s, const double* __restrict__ iw,
                           const double* __restrict__ gridd, int nf, int width, double* __restrict__ gb,
                           double* __restrict__ gx) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const double b = beta[j], qj = q[j], sj = sig[j];
  gb[j] -= qj * sj / (b * b);
  if (gx) {
    const double w = xloc[j] + xw[j] + interp_pre(j, i0s, iw, gridd, nf, width);
    gx[j] += qj * (D[j] + Dloc[j]) + sj * w;
  }
}

// Rows 0 .. nlev - 1 of out = levels a - nlev .. a - 1 of a density ring
// (slot L mod NH), the head of the gradient pass's segment buffer.
__global__ void k_seg_head(int M, int NH, int64_t a, int nlev, const double* __restrict__ hist,
                           double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nlev * M) return;
  const int r = (int)(t / M), j = (int)(t % M);
  out[t] = hist[(int64_t)mod_slot(a - nlev + r, NH) * M + j];
}

// v_j <- v_j / (beta_j / 2): a local sum with the stored beta_j/2-scaled weights
// back to the field value.
__global__ void k_unscale(int M, const double* __restrict__ beta, double* __restrict__ v) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M) v[j] = v[j] / (0.5 * beta[j]);
}

// out[i] = in[idx[i]]
__global__ void k_gather(int n, const int* __restrict__ idx, const double* __restrict__ in, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[idx[i]];
}

// Caller-supplied driving data g (caller order) into the solve's input in
// sorted order, where it enters the right-hand side with a minus sign:
// out[j] = -g[perm[j]].
__global__ void k_drive_gather(int M, const int* __restrict__ perm, const double* __restrict__ g,
                               double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M) out[j] = -g[perm[j]];
}

// out[perm[j]] = in[j]  (sorted -> caller order)
__global__ void k_unsort(int M, const int* __restrict__ perm, const double* __restrict__ in, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M) out[perm[j]] = in[j];
}

// ---------------------------------------------------------------------------
// Batched form: each stage of a level is one launch over a work list of
// (instance, block) items; every item runs the single-instance kernel body
// with its instance's descriptor.  The level index is read from device memory
// so that a whole level can be captured once in a HIP graph and replayed.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) kb_incident(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  const Packets pk{d.npk, 1, d.packets};
  k_incident_body(d.M, (double)(*b.level) * d.dt, d.xs, d.beta, pk, d.pp, 0, d.ginc, w.y);
}

__global__ void __launch_bounds__(512) kb_local(BatchLaunch b, int xcd) {
  const int2 w = b.work[xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  k_local_rhs_body(d.M, d.NQ, d.NH, *b.level, 1, d.NQ, d.nb_start, d.rowbase, d.acx, d.Qc, d.hist, nullptr, d.loc,
                   w.y);
}

// Instances whose lag blocks are short: 8 or 4 lanes per lag.
__global__ void __launch_bounds__(256) kb_local_g8(BatchLaunch b) {
  const int2 w = b.work[xcd_block(blockIdx.x, gridDim.x)];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  k_local_rhs_body<8>(d.M, d.NQ, d.NH, *b.level, 1, d.NQ, d.nb_start, d.rowbase, d.acx, d.Qc, d.hist, nullptr,
                      d.loc, w.y);
}

__global__ void __launch_bounds__(256) kb_local_g4(BatchLaunch b) {
  const int2 w = b.work[xcd_block(blockIdx.x, gridDim.x)];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  k_local_rhs_body<4>(d.M, d.NQ, d.NH, *b.level, 1, d.NQ, d.nb_start, d.rowbase, d.acx, d.Qc, d.hist, nullptr,
                      d.loc, w.y);
}

// On-the-fly local sums (each unordered pair once, p = 8): the block pass over
// (instance, row block) items, then the per-row totals over (instance, 256
// rows) items.
__global__ void __launch_bounds__(1024) kb_local_otf(BatchLaunch b) {
  const int2 w = b.work[xcd_block(blockIdx.x, gridDim.x)];
  if (w.x < 0) return;   // block-uniform
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  k_local_otf_sym_body<8>(d.M, d.NH, d.NQ, *b.level, d.otf_up_end, d.otf_blk_end, d.otf_part_off, d.xs, d.hist, 1,
                          d.dt, d.delta, d.W, d.ngl, d.otf_na, d.otf_nw, d.phitab, d.otf_rowacc, d.otf_part, w.y);
}

__global__ void __launch_bounds__(256) kb_local_otf_reduce(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  k_local_otf_reduce_body(d.M, d.otf_nblk, 1, d.otf_blk_end, d.otf_part_off, d.otf_rowacc, d.otf_part, d.half_beta,
                          d.loc, w.y);
}

// Weights stored once per unordered pair (lags >= 1 in one pass, as in a
// plan's on-the-fly schedule): the rows over (instance, block of 4 rows)
// items, then the per-row totals over (instance, 64 rows) items, scaled by
// beta_j / 2 into the instance's local sum.
__global__ void __launch_bounds__(256) kb_local_sym(BatchLaunch b) {
  const int2 w = b.work[xcd_block(blockIdx.x, gridDim.x)];
  if (w.x < 0) return;   // block-uniform
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  if (d.sym_spl == 2)
    k_local_sym_rows_body<2>(d.M, d.NH, d.NQ, *b.level, 1, d.otf_up_end, d.hist, d.sym_rb, d.sym_acx, d.sym_q,
                             d.sym_upb, d.otf_rowacc, d.sym_colpart, w.y);
  else
    k_local_sym_rows_body<1>(d.M, d.NH, d.NQ, *b.level, 1, d.otf_up_end, d.hist, d.sym_rb, d.sym_acx, d.sym_q,
                             d.sym_upb, d.otf_rowacc, d.sym_colpart, w.y);
}

__global__ void __launch_bounds__(64 * kReduceWaves) kb_local_sym_reduce(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;
  k_local_sym_reduce_body(d.M, d.sym_cov, d.sym_upb, d.otf_rowacc, d.sym_colpart, d.half_beta, d.loc, w.y);
}

// Type-1 spreading as its own pass: a work item is 256 consecutive cells of
// one instance's fine grid (one thread per cell, coalesced), written to the
// instance's spread grid for kb_hist_a(from_grid = 1).
__global__ void __launch_bounds__(256) kb_spread_grid(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;
  const int cell = w.y * 256 + (int)threadIdx.x;
  if (cell >= d.nf) return;
  const double* sig = d.hist + (int64_t)mod_slot(*b.level - 1, d.NH) * d.M;
  d.gsp[cell] = spread_cell(cell, sig, d.M, d.cstart, d.ccount, d.swoff, d.sw);
}

// Row pass of the fine-grid transform; from_grid = 0 spreads the row's cells
// itself, 1 reads them from the spread grid.
__global__ void __launch_bounds__(256) kb_hist_a(BatchLaunch b, int from_grid) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  const ExtraSources none{nullptr, 0, nullptr, nullptr, nullptr, nullptr};
  if (from_grid) {
    k_hist_a_body(d.f2, d.n1, nullptr, 0, nullptr, nullptr, nullptr, nullptr, d.tw, d.T1, none, w.y, d.gsp);
    return;
  }
  const double* sig = d.hist + (int64_t)mod_slot(*b.level - 1, d.NH) * d.M;
  k_hist_a_body(d.f2, d.n1, sig, d.M, d.cstart, d.ccount, d.swoff, d.sw, d.tw, d.T1, none, w.y);
}

__global__ void __launch_bounds__(512) kb_hist_b(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  k_hist_b_body(0, d.f1, d.n2, d.K, d.W, *b.level, d.npos, d.T1, d.tw, d.tw1, d.dk1, d.dk2, d.pk, d.qk, d.rot, d.ring,
                d.alpha, d.dalpha, d.ybuf, d.V, kFirGroups, w.y);
}

__global__ void __launch_bounds__(256) kb_hist_c(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  k_hist_c_body(d.f2, d.n1, d.V, d.tw, (double2*)d.grid2, w.y);
}

__global__ void __launch_bounds__(256) kb_solve_direct(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  double* slot = d.hist + (int64_t)mod_slot(*b.level, d.NH) * d.M;
  k_solve_direct_body(d.M, d.dt_g0, d.dt_n, d.dt_p0, d.pt_cs, d.pt_cn, d.pt_inv, d.inv, d.ginc, d.loc, d.i0s, d.iw,
                      d.beta, d.grid2, d.nf, d.width, slot, nullptr, nullptr, w.y);
}

__global__ void __launch_bounds__(256) kb_solve(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  double* slot = d.hist + (int64_t)mod_slot(*b.level, d.NH) * d.M;
  k_solve_body(d.M, d.iters, d.ext_max, d.tile_r0, d.tile_el, d.tile_g0, d.tile_left, d.tile_n, d.srow_g,
               d.srow_dinv, d.srow_ptr, d.scol, d.sval, d.ginc, d.loc, d.i0s, d.iw, d.beta, d.grid2, d.nf, d.width,
               slot, nullptr, nullptr, w.y);
}

__global__ void __launch_bounds__(256) kb_solve_rhs(BatchLaunch b) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  double* slot = d.hist + (int64_t)mod_slot(*b.level, d.NH) * d.M;
  k_solve_rhs_body(d.M, d.ginc, d.loc, d.beta, d.i0s, d.iw, d.grid2, d.nf, d.width, d.g_dinv, d.g_rhs,
                   d.iters > 1 ? d.g_xa : slot, w.y);
}

// Sweep `it` (1-based) of the instances whose sweep count exceeds it; the
// buffers alternate as in the single-instance solve and the last sweep writes
// the history slot.
__global__ void __launch_bounds__(256) kb_jacobi_sweep(BatchLaunch b, int it) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  if (it >= d.iters) return;
  double* slot = d.hist + (int64_t)mod_slot(*b.level, d.NH) * d.M;
  const double* xin = (it & 1) ? d.g_xa : d.g_xb;
  double* xout = (it == d.iters - 1) ? slot : ((it & 1) ? d.g_xb : d.g_xa);
  k_jacobi_sweep_body(d.M, d.g_ptr, d.g_col, d.g_val, d.g_dinv, d.g_rhs, xin, xout, nullptr, nullptr, w.y);
}

// The same sweep with one wavefront per row (4 rows per block), for instances
// whose rows hold many nearby sources.
__global__ void __launch_bounds__(256) kb_jacobi_sweep_wave(BatchLaunch b, int it) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  if (it >= d.iters) return;
  double* slot = d.hist + (int64_t)mod_slot(*b.level, d.NH) * d.M;
  const double* xin = (it & 1) ? d.g_xa : d.g_xb;
  double* xout = (it == d.iters - 1) ? slot : ((it & 1) ? d.g_xb : d.g_xa);
  k_jacobi_sweep_wave_body(d.M, d.g_ptr, d.g_col, d.g_val, d.g_dinv, d.g_rhs, xin, xout, nullptr, nullptr, w.y);
}

// Receivers of every instance at the level being computed: instance i writes
// row (*level - *level0) of uout[i] ([levels][R_i]; NULL: no output).
__global__ void __launch_bounds__(256) kb_receivers(BatchLaunch b, double* const* __restrict__ uout,
                                                    const int64_t* __restrict__ level0) {
  const int2 w = b.work[blockIdx.x];
  if (w.x < 0) return;
  double* out = uout[w.x];
  if (!out) return;
  const InstDesc& d = b.desc[w.x];
  if (*b.level >= d.end) return;   // the instance has marched its own levels (block-uniform)
  const int64_t L = *b.level;
  k_receivers_body(d.R, d.M, d.NQ, d.NH, L, d.rnb_start, d.rnb_count, d.rqoff, d.Qr, d.hist, d.ri0s, d.riw,
                   d.grid2, d.nf, d.width, out + (L - *level0) * d.R, w.y);
}

__global__ void kb_advance(int64_t* level) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *level += 1;
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

__global__ void k_ring_io(int64_t K, int W, int64_t L, int n1, int n2, int64_t npos, int to_user,
                          double2* __restrict__ ring, double2* __restrict__ user) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)W * (K + 1)) return;
  const int m = (int)(t / (K + 1));
  const int64_t k = t % (K + 1);
  const int slot = mod_slot(L - 2 - m, W);
  double2* r = ring + (int64_t)slot * npos + mode_pos(k, n1, n2);
  double2* u = user + (int64_t)m * (K + 1) + k;
  if (to_user) *u = *r;
  else *r = *u;
}

// alpha or alpha' between the position order and the caller's k order.
__global__ void k_modes_io(int64_t K, int n1, int n2, int to_user, double2* __restrict__ a,
                           double2* __restrict__ user) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > K) return;
  double2* r = a + mode_pos(k, n1, n2);
  if (to_user) user[k] = *r;
  else *r = user[k];
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_int(int* __restrict__ p, int64_t n, int v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Sets *flag to 1 when any of a[0 .. na) or b[0 .. nb) is NaN or infinite
// (grid-stride loop; b may be NULL with nb = 0).
__global__ void k_check_finite(const double* __restrict__ a, int64_t na, const double* __restrict__ b, int64_t nb,
                               int* __restrict__ flag) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride)
    bad |= !isfinite(i < na ? a[i] : b[i - na]);
  if (bad) atomicOr(flag, 1);
}

}  // namespace wfp
