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

// Extra spreading sources (the receivers in the gradient pass): values val[i]
// at sorted positions i = 0..n-1 with per-cell ranges and weights like the
// scatterers'.  val == nullptr means none.
struct ExtraSources {
  const double* val;
  int n;
  const int* cstart;
  const int* ccount;
  const int64_t* woff;
  const double* w;
};

struct Packets {
  int n;
  int periodic;
  const double* p;            // [n][5] amp, centre, width, omega, phase
};

// ---- set-up kernels ----
__global__ void k_pq_tables(int64_t K, int W, int ng, double dt, const double* __restrict__ dphi_tab,
                            const double* __restrict__ ddphi_tab, const double* __restrict__ mu,
                            const double* __restrict__ wmu, int n1, int n2, int64_t npos,
                            double* __restrict__ pk, double* __restrict__ qk, double* __restrict__ rot);

template <int P>
__global__ void k_local_weights(int nrows, const double* __restrict__ xt,
                                const double* __restrict__ xs, int M,
                                const int* __restrict__ nb_start, const int* __restrict__ nb_count,
                                const int64_t* __restrict__ qoff, const double* __restrict__ rowscale,
                                int periodic, double dt, double delta, int W, int NQ, int ngl,
                                const double* __restrict__ glz, const double* __restrict__ glw,
                                const double* __restrict__ cheb_phi, const double* __restrict__ cheb_g,
                                int ncheb, int deriv,
                                const double* __restrict__ lagw, const int64_t* __restrict__ pbase,
                                signed char* __restrict__ mlo, int nq_out, double* __restrict__ Q);

constexpr int kPhiPieces = 512, kPhiDeg = 5;
constexpr int kOtfRows = 16, kOtfChunk = 256;
// wavefronts of a pair-once reduce workgroup (64 rows, one per lane)
constexpr int kReduceWaves = 16;
// sources per LDS chunk of the on-the-fly derivative local sums
constexpr int kOtfDerivChunk = 112;
constexpr int kMaxOtfLags = 48;      // lags 1 .. NQ - 1 of a row staged by the symmetric local sum
template <int P>
__global__ void k_local_otf_sym(int M, int NH, int NQ, int64_t L, const int* __restrict__ up_end,
                                const int* __restrict__ blk_end, const int64_t* __restrict__ part_off,
                                int nblk_rows, const double* __restrict__ xs, const double* __restrict__ hist,
                                int periodic, double dt, double delta, int W, int ngl,
                                const double* __restrict__ na, const double* __restrict__ nw,
                                const double* __restrict__ phitab, double* __restrict__ rowacc,
                                double* __restrict__ part);
template <int SPL>
__global__ void k_local_sym_rows(int M, int NH, int NQ, int64_t L, int mfirst, const int* __restrict__ up_end,
                                 const double* __restrict__ hist, const int64_t* __restrict__ rb,
                                 const uint2* __restrict__ sacx, const double* __restrict__ Qs,
                                 const int64_t* __restrict__ upb, double* __restrict__ rowacc,
                                 double* __restrict__ colpart);
template <int P>
__global__ void k_local_otf_deriv2(int M, int NH, int NQ, const int* __restrict__ up_end,
                                   const int* __restrict__ blk_end, const int64_t* __restrict__ part_off,
                                   int nblk_rows, const double* __restrict__ xs, const double* __restrict__ h1,
                                   int64_t r1, const double* __restrict__ h2, int64_t L2, int periodic, double dt,
                                   double delta, int W, int ngl, const double* __restrict__ na,
                                   const double* __restrict__ nw, const double* __restrict__ phitab,
                                   double* __restrict__ row1, double* __restrict__ row2, double* __restrict__ row3,
                                   double* __restrict__ part1, double* __restrict__ part2, double* __restrict__ part3);
template <int SPL>
__global__ void k_local_sym_deriv2(int M, int NQ, int NH, const int* __restrict__ up_end,
                                   const double* __restrict__ h1, int64_t r1, const double* __restrict__ h2,
                                   int64_t L2, const int64_t* __restrict__ rb, const uint2* __restrict__ sacx,
                                   const double* __restrict__ Qs, const int64_t* __restrict__ upb,
                                   double* __restrict__ row1, double* __restrict__ row2, double* __restrict__ col1,
                                   double* __restrict__ col2);
__global__ void k_local_sym_reduce(int M, const int2* __restrict__ cov, const int64_t* __restrict__ upb,
                                   const double* __restrict__ rowacc, const double* __restrict__ colpart,
                                   const double* __restrict__ scale, double* __restrict__ out);
__global__ void k_local_sym_lag1(int M, int NQ, int NH, int64_t L, int periodic, int kmax,
                                 const int64_t* __restrict__ rb, const uint2* __restrict__ sacx,
                                 const double* __restrict__ Qs, const double* __restrict__ hist,
                                 const double* __restrict__ scale, const double* __restrict__ base,
                                 double* __restrict__ out);
__global__ void k_local_otf_reduce(int M, int nblk_rows, int periodic, const int* __restrict__ blk_end,
                                   const int64_t* __restrict__ part_off, const double* __restrict__ rowacc,
                                   const double* __restrict__ part, const double* __restrict__ scale,
                                   double* __restrict__ out);

__global__ void k_row_ranges(int M, int NQ, const int* __restrict__ nb_count, const int64_t* __restrict__ pbase,
                             const signed char* __restrict__ mlo, unsigned* __restrict__ ac);
__global__ void k_pack_weights(int M, int NQ, int m0, const int* __restrict__ nb_count,
                               const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                               const unsigned* __restrict__ ac, const int64_t* __restrict__ rowbase,
                               double* __restrict__ Qc);
__global__ void k_gather_solve(int64_t ne, const int64_t* __restrict__ eq, const double* __restrict__ Q,
                               double* __restrict__ ev, int64_t nr, const int64_t* __restrict__ rq,
                               double* __restrict__ rdinv);

__global__ void k_row_contraction(int M, const int* __restrict__ nb_start,
                                  const int* __restrict__ nb_count, const int64_t* __restrict__ qoff,
                                  const double* __restrict__ Q, const int* __restrict__ near_start,
                                  const int* __restrict__ near_count, double* __restrict__ out);

__global__ void k_count_nonzero(int M, int NQ, const int* __restrict__ nb_count,
                                const int64_t* __restrict__ qoff, const double* __restrict__ Q,
                                unsigned long long* __restrict__ out);

// ---- per-level kernels ----
__global__ void k_local_rhs(int M, int NQ, int NH, int64_t L, int m0, int m1, const int* __restrict__ nb_start,
                            const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx,
                            const double* __restrict__ Qc, const double* __restrict__ hist,
                            const double* __restrict__ addin, double* __restrict__ loc,
                            double* __restrict__ loc2, int nsplit);
__global__ void k_local_rhs_g8(int M, int NQ, int NH, int64_t L, int m0, int m1, const int* __restrict__ nb_start,
                               const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx,
                               const double* __restrict__ Qc, const double* __restrict__ hist,
                               const double* __restrict__ addin, double* __restrict__ loc);
__global__ void k_local_rhs_g4(int M, int NQ, int NH, int64_t L, int m0, int m1, const int* __restrict__ nb_start,
                               const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx,
                               const double* __restrict__ Qc, const double* __restrict__ hist,
                               const double* __restrict__ addin, double* __restrict__ loc);
__global__ void k_local_lag1(int M, int NQ, int NH, int64_t L, const int* __restrict__ nb_start,
                             const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx,
                             const double* __restrict__ Qc, const double* __restrict__ hist,
                             const double* __restrict__ addin, const double* __restrict__ addin2, int nadd2,
                             double* __restrict__ loc);
__global__ void k_incident(int M, double t, const double* __restrict__ xs, const double* __restrict__ beta,
                           Packets pk, int pp, int deriv, double* __restrict__ ginc);
__global__ void k_incident_levels(int M, int64_t L0, double dt, const double* __restrict__ xs,
                                  const double* __restrict__ beta, Packets pk, int pp, double* __restrict__ out);
__global__ void k_spread_weights(int nf, double hf, double inv_alpha, double beta_es, const double* __restrict__ xs,
                                 int M, const int* __restrict__ cstart, const int* __restrict__ ccount,
                                 const int64_t* __restrict__ woff, double* __restrict__ w);
__global__ void k_interp_weights(int n, int nf, double hf, double inv_alpha, double beta_es, int width,
                                 const double* __restrict__ x, int* __restrict__ i0s, double* __restrict__ w);

__global__ void k_solve(int M, int iters, int ext_max, const int* __restrict__ tile_r0,
                        const int* __restrict__ tile_el, const int* __restrict__ tile_g0,
                        const int* __restrict__ tile_left, const int* __restrict__ tile_n,
                        const int* __restrict__ rg, const double* __restrict__ rdinv,
                        const int* __restrict__ rptr, const int* __restrict__ ecol,
                        const double* __restrict__ ev, const double* __restrict__ ginc,
                        const double* __restrict__ loc, const int* __restrict__ i0s,
                        const double* __restrict__ iw, const double* __restrict__ beta,
                        const double* __restrict__ grid2, int nf, int width, double* __restrict__ sig_out,
                        double* __restrict__ save_row, const int* __restrict__ perm);

__global__ void k_solve_rhs(int M, const double* __restrict__ ginc, const double* __restrict__ loc,
                            const double* __restrict__ beta, const int* __restrict__ i0s,
                            const double* __restrict__ iw, const double* __restrict__ grid2, int nf, int width,
                            const double* __restrict__ dinv, double* __restrict__ rhs, double* __restrict__ x);
__global__ void k_jacobi_sweep(int M, const int* __restrict__ ptr, const int* __restrict__ col,
                               const double* __restrict__ val, const double* __restrict__ dinv,
                               const double* __restrict__ rhs, const double* __restrict__ xin,
                               double* __restrict__ xout, double* __restrict__ save_row,
                               const int* __restrict__ perm);
__global__ void k_jacobi_sweep_wave(int M, const int* __restrict__ ptr, const int* __restrict__ col,
                                    const double* __restrict__ val, const double* __restrict__ dinv,
                                    const double* __restrict__ rhs, const double* __restrict__ xin,
                                    double* __restrict__ xout, double* __restrict__ save_row,
                                    const int* __restrict__ perm);
__global__ void k_solve_direct(int M, const int* __restrict__ dt_g0, const int* __restrict__ dt_n,
                               const int* __restrict__ dt_p0, const int* __restrict__ pt_cs,
                               const int* __restrict__ pt_cn, const int64_t* __restrict__ pt_inv,
                               const double* __restrict__ inv, const double* __restrict__ ginc,
                               const double* __restrict__ loc, const int* __restrict__ i0s,
                               const double* __restrict__ iw, const double* __restrict__ beta,
                               const double* __restrict__ grid2, int nf, int width,
                               double* __restrict__ sig_out, double* __restrict__ save_row,
                               const int* __restrict__ perm);
__global__ void k_receivers(int M, int NQ, int NH, int64_t L, const int* __restrict__ nb_start,
                            const int* __restrict__ nb_count, const int64_t* __restrict__ qoff,
                            const double* __restrict__ Q, const double* __restrict__ hist, const int* __restrict__ i0s,
                            const double* __restrict__ iw, const double* __restrict__ grid2, int nf, int width,
                            double* __restrict__ out);

// ---- history part as three kernels (four-step transform, n = n1 n2) ----
__global__ void k_hist_a(FftPlan f2, int n1, const double* __restrict__ sig, int M,
                         const int* __restrict__ cstart, const int* __restrict__ ccount,
                         const int64_t* __restrict__ woff, const double* __restrict__ sw,
                         const double2* __restrict__ tw, double2* __restrict__ T1, ExtraSources ex);
// FIR taps split over G groups whose partial sums meet in LDS ([G][2 n1] double4)
__global__ void k_hist_b(int mode, FftPlan f1, int n2, int64_t K, int W, int64_t L, int64_t npos,
                         const double2* __restrict__ T1, const double2* __restrict__ tw,
                         const double2* __restrict__ tw1, const double* __restrict__ dk1, const double* __restrict__ dk2,
                         const double* __restrict__ pk, const double* __restrict__ qk,
                         const double* __restrict__ rot, double2* __restrict__ ring,
                         double2* __restrict__ alpha, double2* __restrict__ dalpha, double2* __restrict__ y,
                         double2* __restrict__ V, int G, int vcol);
__global__ void k_hist_c(FftPlan f2, int n1, const double2* __restrict__ V, const double2* __restrict__ tw,
                         double2* __restrict__ grid2);
// the same row passes with 1024 threads, for rows of more than 1024 butterflies per stage at 256
__global__ void k_hist_a_wide(FftPlan f2, int n1, const double* __restrict__ grid, const double2* __restrict__ tw,
                              double2* __restrict__ T1);
// type-1 spreading, one thread per fine-grid cell (feeds k_hist_a_wide)
__global__ void k_spread_grid(int nf, const double* __restrict__ sig, int M, const int* __restrict__ cstart,
                              const int* __restrict__ ccount, const int64_t* __restrict__ woff,
                              const double* __restrict__ sw, ExtraSources ex, double* __restrict__ grid);
__global__ void k_hist_c_wide(FftPlan f2, int n1, const double2* __restrict__ V, const double2* __restrict__ tw,
                              double2* __restrict__ grid2);

// ---- free-space radiation boundary projection ----
__global__ void k_rbc_to_grid(FftPlan fp, int64_t K, int n1, int n2, const double2* __restrict__ alpha,
                              const double2* __restrict__ dalpha, const double2* __restrict__ tw,
                              double2* __restrict__ gu, double2* __restrict__ gv);
__global__ void k_rbc_to_modes(FftPlan fp, int64_t K, int n1, int n2, int W, double h, double delta_s,
                               const double* __restrict__ cheb_phi, const double* __restrict__ cheb_g,
                               int ncheb, const double* __restrict__ gu, const double* __restrict__ gv,
                               const double2* __restrict__ tw, const double* __restrict__ dk2,
                               double2* __restrict__ alpha, double2* __restrict__ dalpha,
                               double2* __restrict__ y);
// long grids: pack, the length-K transform in two passes over workgroups (K = a b), unpack
__global__ void k_rbc_grid_pack(int64_t K, int n1, int n2, const double2* __restrict__ alpha,
                                const double2* __restrict__ dalpha, const double2* __restrict__ tw,
                                double2* __restrict__ z);
__global__ void k_rbc_fft_pass1(FftPlan fb, int a, int64_t K, const double2* __restrict__ tw,
                                const double2* __restrict__ z, double2* __restrict__ T);
__global__ void k_rbc_fft_pass2(FftPlan fa, int b, int64_t K, const double2* __restrict__ tw,
                                const double2* __restrict__ T, double2* __restrict__ out0,
                                double2* __restrict__ out1, int conj_out);
__global__ void k_rbc_modes_pack(int64_t K, int W, double h, double delta_s, const double* __restrict__ cheb_phi,
                                 const double* __restrict__ cheb_g, int ncheb, const double* __restrict__ gu,
                                 const double* __restrict__ gv, double2* __restrict__ z);
__global__ void k_rbc_modes_unpack(int64_t K, int n1, int n2, const double2* __restrict__ X,
                                   const double2* __restrict__ tw, const double* __restrict__ dk2,
                                   double2* __restrict__ alpha, double2* __restrict__ dalpha,
                                   double2* __restrict__ y);

// ---- gradient pass ----
__global__ void k_deriv_y(int64_t K, int n1, int n2, const double2* __restrict__ alpha,
                          const double* __restrict__ dk2, double2* __restrict__ y);
__global__ void k_adj_drive(int M, int R, int NQ, int64_t L, int64_t N, const int* __restrict__ ptr,
                            const int* __restrict__ rr, const int* __restrict__ ri,
                            const int64_t* __restrict__ rqoff, const int* __restrict__ rcount,
                            const double* __restrict__ Qr, const double* __restrict__ dQr,
                            const double* __restrict__ e, const double* __restrict__ beta,
                            double* __restrict__ ginc, double* __restrict__ xw);
__global__ void k_fwd_dterm(int M, const double* __restrict__ fprime, const int* __restrict__ i0s,
                            const double* __restrict__ iw, const double* __restrict__ gridd, int nf, int width,
                            double* __restrict__ D);
__global__ void k_adj_grad(int M, const double* __restrict__ q, const double* __restrict__ sig,
                           const double* __restrict__ beta, const double* __restrict__ D,
                           const double* __restrict__ Dloc, const double* __restrict__ xloc,
                           const double* __restrict__ xw, const int* __restrict__ i0s, const double* __restrict__ iw,
                           const double* __restrict__ gridd, int nf, int width, double* __restrict__ gb,
                           double* __restrict__ gx);
__global__ void k_local_deriv2(int M, int NQ, int NH, const int* __restrict__ nb_start,
                               const int64_t* __restrict__ rowbase, const uint2* __restrict__ acx,
                               const double* __restrict__ Qc, const double* __restrict__ h1, int64_t r1,
                               const double* __restrict__ h2, int64_t L2, double* __restrict__ out1,
                               double* __restrict__ out2);
__global__ void k_seg_head(int M, int NH, int64_t a, int nlev, const double* __restrict__ hist,
                           double* __restrict__ out);
__global__ void k_unscale(int M, const double* __restrict__ beta, double* __restrict__ v);
__global__ void k_gather(int n, const int* __restrict__ idx, const double* __restrict__ in, double* __restrict__ out);
__global__ void k_drive_gather(int M, const int* __restrict__ perm, const double* __restrict__ g,
                               double* __restrict__ out);
__global__ void k_unsort(int M, const int* __restrict__ perm, const double* __restrict__ in, double* __restrict__ out);

// ---- batched form: one launch per stage over an (instance, block) work list ----
// Everything the level kernels of one instance read.
struct InstDesc {
  int M, NQ, NH, W, nf, width, n1, n2, iters, npk, pp, ext_max, global_solve;
  int64_t K, npos;
  int64_t end;                 // the instance computes levels L < end (its own N_t)
  double dt;
  FftPlan f1, f2;
  const double *xs, *beta, *packets;
  const int* nb_start;
  const int64_t* rowbase;
  const uint2* acx;
  const double* Qc;
  double *hist, *loc, *ginc;
  const int *cstart, *ccount;
  const int64_t* swoff;
  const double* sw;
  const double2* tw;
  const double2* tw1;
  double2 *T1, *V;
  double* grid2;
  double* gsp;                 // fine grid spread by a separate pass (batched spread_pass 1)
  const double *dk1, *dk2, *pk, *qk, *rot;
  double2 *ring, *alpha, *dalpha, *ybuf;
  const int *dt_g0, *dt_n, *dt_p0, *pt_cs, *pt_cn;
  const int64_t* pt_inv;
  const double* inv;
  const int *tile_r0, *tile_el, *tile_g0, *tile_left, *tile_n, *srow_g, *srow_ptr, *scol;
  const double *srow_dinv, *sval;
  const int* i0s;
  const double* iw;
  const int *g_ptr, *g_col;
  const double *g_val, *g_dinv;
  double *g_rhs, *g_xa, *g_xb;
  // local weights on the fly (p = 8), each unordered pair once
  int otf, ngl;
  double delta;
  const int* nb_count;
  const double *otf_z, *otf_w, *phitab, *half_beta;
  const int *otf_up_end, *otf_blk_end;
  const int64_t* otf_part_off;
  int otf_nblk;
  const double *otf_na, *otf_nw;
  double *otf_part, *otf_rowacc;
  // weights stored once per unordered pair (otf_up_end, otf_rowacc shared)
  int sym, sym_spl;
  const int64_t* sym_rb;
  const uint2* sym_acx;
  const double* sym_q;
  const int64_t* sym_upb;
  double* sym_colpart;
  const int2* sym_cov;
  // receivers
  int R;
  const int *rnb_start, *rnb_count, *ri0s;
  const int64_t* rqoff;
  const double *Qr, *riw;
};

// Work item (instance, block within the instance); instance < 0 pads the list.
struct BatchLaunch {
  const InstDesc* desc;
  const int2* work;
  const int64_t* level;   // the level all instances compute (device)
};

__global__ void kb_incident(BatchLaunch b);
__global__ void kb_receivers(BatchLaunch b, double* const* __restrict__ uout, const int64_t* __restrict__ level0);
__global__ void kb_local(BatchLaunch b, int xcd);
__global__ void kb_local_g8(BatchLaunch b);
__global__ void kb_local_g4(BatchLaunch b);
__global__ void kb_local_otf(BatchLaunch b);
__global__ void kb_local_otf_reduce(BatchLaunch b);
__global__ void kb_local_sym(BatchLaunch b);
__global__ void kb_local_sym_reduce(BatchLaunch b);
__global__ void kb_spread_grid(BatchLaunch b);
__global__ void kb_hist_a(BatchLaunch b, int from_grid);
__global__ void kb_hist_b(BatchLaunch b);
__global__ void kb_hist_c(BatchLaunch b);
__global__ void kb_solve_direct(BatchLaunch b);
__global__ void kb_solve(BatchLaunch b);
__global__ void kb_solve_rhs(BatchLaunch b);
__global__ void kb_jacobi_sweep(BatchLaunch b, int it);
__global__ void kb_jacobi_sweep_wave(BatchLaunch b, int it);
__global__ void kb_advance(int64_t* level);

// ---- state movement ----
__global__ void k_hist_io(int M, int NH, int64_t L, int to_user, double* __restrict__ hist,
                          double* __restrict__ user, const int* __restrict__ perm);
__global__ void k_ring_io(int64_t K, int W, int64_t L, int n1, int n2, int64_t npos, int to_user,
                          double2* __restrict__ ring, double2* __restrict__ user);
__global__ void k_modes_io(int64_t K, int n1, int n2, int to_user, double2* __restrict__ a,
                           double2* __restrict__ user);
__global__ void k_fill(double* __restrict__ p, int64_t n, double v);
__global__ void k_fill_int(int* __restrict__ p, int64_t n, int v);
__global__ void k_check_finite(const double* __restrict__ a, int64_t na, const double* __restrict__ b, int64_t nb,
                               int* __restrict__ flag);

}  // namespace wfp
