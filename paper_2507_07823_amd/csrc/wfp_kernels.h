// Device kernels of the WFP march (gfx950, FP64).  Internal header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wfp {

constexpr int kMaxFftStages = 24;
constexpr int kFftThreads = 1024;
constexpr int kFftMaxB = 4;          // butterflies per thread per stage
constexpr int kMaxP = 12;            // largest supported interpolation order
constexpr int kRowThreads = 256;     // 4 wavefronts -> 4 target rows per block

struct FftPlan {
  int n;                      // complex length (half the real length)
  int nst;
  int radix[kMaxFftStages];
};

struct Packets {
  int n;
  int periodic;
  const double* p;            // [n][5] amp, centre, width, omega, phase
};

// ---- set-up kernels ----
__global__ void k_pq_tables(int64_t K, int W, int ng, double dt, const double* __restrict__ dphi_tab,
                            const double* __restrict__ ddphi_tab, const double* __restrict__ mu,
                            const double* __restrict__ wmu, double* __restrict__ pk,
                            double* __restrict__ qk, double* __restrict__ rot);

template <int P>
__global__ void k_local_weights(int nrows, const double* __restrict__ xt,
                                const double* __restrict__ xs, int M,
                                const int* __restrict__ nb_start, const int* __restrict__ nb_count,
                                const int64_t* __restrict__ qoff, const double* __restrict__ rowscale,
                                int periodic, double dt, double delta, int W, int NQ, int ngl,
                                const double* __restrict__ glz, const double* __restrict__ glw,
                                const double* __restrict__ cheb_phi, int ncheb,
                                const double* __restrict__ lagw, double* __restrict__ Q);

__global__ void k_row_contraction(int M, const int* __restrict__ nb_start,
                                  const int* __restrict__ nb_count, const int64_t* __restrict__ qoff,
                                  const double* __restrict__ Q, const int* __restrict__ near_start,
                                  const int* __restrict__ near_count, double* __restrict__ out);

// ---- per-level kernels ----
__global__ void k_spread(int nf, double hf, double inv_alpha, double beta_es,
                         const double* __restrict__ xs, const double* __restrict__ sig, int M,
                         const int* __restrict__ cstart, const int* __restrict__ ccount,
                         double* __restrict__ grid);

__global__ void k_fft_r2c(FftPlan fp, const double2* __restrict__ grid, const double2* __restrict__ tw,
                          int tws, double2* __restrict__ zout);

__global__ void k_modes(int64_t K, int W, int nfh, int64_t L, const double2* __restrict__ z,
                        const double2* __restrict__ tw, const double* __restrict__ dk1,
                        const double* __restrict__ dk2, const double* __restrict__ pk,
                        const double* __restrict__ qk, const double* __restrict__ rot,
                        double2* __restrict__ ring, double2* __restrict__ alpha,
                        double2* __restrict__ dalpha, double2* __restrict__ y);

__global__ void k_fft_c2r(FftPlan fp, int64_t K, const double2* __restrict__ y,
                          const double2* __restrict__ tw, int tws, double2* __restrict__ grid_out);

__global__ void k_local_rhs(int M, int NQ, int NH, int64_t L, double t,
                            const double* __restrict__ xs, const double* __restrict__ beta,
                            const int* __restrict__ nb_start, const int* __restrict__ nb_count,
                            const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                            const double* __restrict__ hist, const double* __restrict__ grid2, int nf,
                            double hf, double inv_alpha, double beta_es, int width, Packets pk,
                            double* __restrict__ rhs);

__global__ void k_jacobi(int M, int T, int iters, int ext_max, const int* __restrict__ ext_start,
                         const int* __restrict__ ext_len, const int* __restrict__ nb_start,
                         const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                         const int* __restrict__ near_start, const int* __restrict__ near_count,
                         const double* __restrict__ rhs, double* __restrict__ sig_out,
                         double* __restrict__ save_row, const int* __restrict__ perm);

__global__ void k_receivers(int R, int M, int NQ, int NH, int64_t L, const double* __restrict__ xr,
                            const int* __restrict__ nb_start, const int* __restrict__ nb_count,
                            const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                            const double* __restrict__ hist, const double* __restrict__ grid2, int nf,
                            double hf, double inv_alpha, double beta_es, int width,
                            double* __restrict__ out);

// ---- free-space radiation boundary projection ----
__global__ void k_rbc_to_grid(FftPlan fp, int64_t K, const double2* __restrict__ alpha,
                              const double2* __restrict__ dalpha, const double2* __restrict__ tw,
                              double2* __restrict__ gu, double2* __restrict__ gv);
__global__ void k_rbc_to_modes(FftPlan fp, int64_t K, int W, double h, double delta_s,
                               const double* __restrict__ cheb_phi, const double* __restrict__ cheb_g,
                               int ncheb, const double* __restrict__ gu, const double* __restrict__ gv,
                               const double2* __restrict__ tw, const double* __restrict__ dk2,
                               double2* __restrict__ alpha, double2* __restrict__ dalpha,
                               double2* __restrict__ y);

// ---- state movement ----
__global__ void k_hist_io(int M, int NH, int64_t L, int to_user, double* __restrict__ hist,
                          double* __restrict__ user, const int* __restrict__ perm);
__global__ void k_ring_io(int64_t K, int W, int64_t L, int to_user, double2* __restrict__ ring,
                          double2* __restrict__ user);
__global__ void k_fill(double* __restrict__ p, int64_t n, double v);

}  // namespace wfp
