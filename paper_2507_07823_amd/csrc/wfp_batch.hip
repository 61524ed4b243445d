// Batched form: many independent periodic problems marched in lockstep, each
// stage of a level one launch over an (instance, block) work list, the whole
// level captured once in a HIP graph (the level index lives on the device).
// Each instance is an ordinary plan (wfp_plan_create); the batch only adds the
// descriptor table, the work lists, the graph and the launch-shape autotuner.
#include "wfp_internal.h"

struct wfp_batch {
  int device = 0;
  hipStream_t user_stream = nullptr;   // the caller's stream (ordering only)
  hipStream_t bs = nullptr;            // the batch's own stream (graph capture)
  hipStream_t bs2 = nullptr;           // second branch of the captured level (history chain)
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr, ev_join = nullptr;
  std::vector<wfp_plan*> plans;
  int64_t level = 0;
  int64_t* level_d = nullptr;
  InstDesc* desc_d = nullptr;
  std::vector<InstDesc> desc_h;        // host copy of the descriptor table
  std::vector<int64_t> ends;           // per instance: levels L < ends[i] are computed
  // work lists (device) and their lengths
  int2 *wl_inc = nullptr, *wl_loc4 = nullptr, *wl_loc8 = nullptr, *wl_a = nullptr, *wl_b = nullptr,
       *wl_c = nullptr, *wl_dir = nullptr, *wl_til = nullptr, *wl_rows = nullptr, *wl_otf = nullptr,
       *wl_swt = nullptr, *wl_sww = nullptr, *wl_g8 = nullptr, *wl_g4 = nullptr, *wl_rcv = nullptr,
       *wl_otfr = nullptr, *wl_sp = nullptr, *wl_sym = nullptr, *wl_symr = nullptr;
  int n_otfr = 0, n_sp = 0, n_sym = 0, n_symr = 0;
  int n_inc = 0, n_loc4 = 0, n_loc8 = 0, n_a = 0, n_b = 0, n_c = 0, n_dir = 0, n_til = 0, n_rows = 0, n_otf = 0,
      n_swt = 0, n_sww = 0, n_g8 = 0, n_g4 = 0, n_rcv = 0;
  // receiver outputs of the current run: per instance a device pointer (or
  // NULL) and the level the run started at, read by the captured level
  double** uout_d = nullptr;
  int64_t* lvl0_d = nullptr;
  bool uout_set = false;
  size_t lds_a = 0, lds_b = 0, lds_c = 0, lds_til = 0, lds_otf = 0;
  // Jacobi sweeps of the global-solve instances, thread per row (swt) or
  // wavefront per row (sww); both lists are ordered by decreasing sweep count,
  // so sweep `it` launches the prefix of cnt_swt[it] (cnt_sww[it]) items
  // whose instances still iterate
  int max_sweeps = 0;
  std::vector<int> cnt_swt, cnt_sww;
  // launch shape of the local sum: rows per block (4 or 8) and the XCD remap
  int loc_rows = 4, loc_xcd = 1;
  // spread tile: 0 = one fine-grid row per workgroup, spread inside the row
  // pass of the transform (cells n1 apart); 1 = 256 consecutive cells per
  // workgroup in a separate coalesced pass, the row pass reading the grid
  int spread_pass = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<void*> owned;
  ~wfp_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (wfp_plan* p : plans) wfp_plan_destroy(p);
    for (void* q : owned) (void)hipFree(q);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (bs2) (void)hipStreamDestroy(bs2);
    if (bs) (void)hipStreamDestroy(bs);
  }
  template <class T>
  T* alloc(size_t n) {
    int64_t dummy = 0;
    T* q = dalloc<T>(n, dummy);
    owned.push_back(q);
    return q;
  }
};

namespace {

InstDesc describe(const wfp_plan* P) {
  InstDesc d{};
  d.M = (int)P->M;
  d.NQ = P->NQ;
  d.NH = P->NH;
  d.W = P->W;
  d.nf = P->nf;
  d.width = P->width;
  d.n1 = P->n1;
  d.n2 = P->n2;
  d.iters = P->iters;
  d.npk = P->npk;
  int pp = 1;
  while (pp < P->npk) pp *= 2;
  d.pp = pp;
  d.ext_max = P->ext_max;
  d.global_solve = P->solve_global ? 1 : 0;
  d.K = P->K;
  d.npos = P->npos;
  d.dt = P->dt;
  d.f1 = P->fft_n1;
  d.f2 = P->fft_n2;
  d.xs = P->xs;
  d.beta = P->beta;
  d.packets = P->packets;
  d.nb_start = P->nb_start;
  d.rowbase = P->rowbase;
  d.acx = P->acx;
  d.Qc = P->Qc;
  d.hist = P->hist;
  d.loc = P->loc;
  d.ginc = P->ginc;
  d.cstart = P->cstart;
  d.ccount = P->ccount;
  d.swoff = P->swoff;
  d.sw = P->sw;
  d.tw = P->tw;
  d.tw1 = P->tw1;
  d.T1 = P->T1;
  d.V = P->V;
  d.grid2 = P->grid2;
  d.gsp = P->gsp;
  d.dk1 = P->dk1;
  d.dk2 = P->dk2;
  d.pk = P->pk;
  d.qk = P->qk;
  d.rot = P->rot;
  d.ring = P->ring;
  d.alpha = P->alpha;
  d.dalpha = P->dalpha;
  d.ybuf = P->ybuf;
  d.dt_g0 = P->dt_g0;
  d.dt_n = P->dt_n;
  d.dt_p0 = P->dt_p0;
  d.pt_cs = P->pt_cs;
  d.pt_cn = P->pt_cn;
  d.pt_inv = P->pt_inv;
  d.inv = P->inv;
  d.tile_r0 = P->tile_r0;
  d.tile_el = P->tile_el;
  d.tile_g0 = P->tile_g0;
  d.tile_left = P->tile_left;
  d.tile_n = P->tile_n;
  d.srow_g = P->srow_g;
  d.srow_ptr = P->srow_ptr;
  d.scol = P->scol;
  d.srow_dinv = P->srow_dinv;
  d.sval = P->sval;
  d.i0s = P->i0s;
  d.iw = P->iw;
  d.g_ptr = P->g_ptr;
  d.g_col = P->g_col;
  d.g_val = P->g_val;
  d.g_dinv = P->g_dinv;
  d.g_rhs = P->g_rhs;
  d.g_xa = P->g_xa;
  d.g_xb = P->g_xb;
  d.otf = P->otf ? 1 : 0;
  d.ngl = P->ngl;
  d.delta = P->delta;
  d.nb_count = P->nb_count;
  d.otf_z = P->otf_z;
  d.otf_w = P->otf_w;
  d.phitab = P->phitab;
  d.half_beta = P->half_beta;
  d.otf_up_end = P->otf_up_end;
  d.otf_blk_end = P->otf_blk_end;
  d.otf_part_off = P->otf_part_off;
  d.otf_nblk = P->otf_nblk;
  d.otf_na = P->otf_na;
  d.otf_nw = P->otf_nw;
  d.otf_part = P->otf_part;
  d.otf_rowacc = P->otf_rowacc;
  d.sym = P->sym_stored ? 1 : 0;
  d.sym_spl = P->sym_spl;
  d.sym_rb = P->sym_rb;
  d.sym_acx = P->sym_acx;
  d.sym_q = P->sym_q;
  d.sym_upb = P->sym_upb;
  d.sym_colpart = P->sym_colpart;
  d.sym_cov = P->sym_cov;
  d.R = (int)P->R;
  d.rnb_start = P->rnb_start;
  d.rnb_count = P->rnb_count;
  d.rqoff = P->rqoff;
  d.Qr = P->Qr;
  d.ri0s = P->ri0s;
  d.riw = P->riw;
  return d;
}

// Work list of (instance, block) items, padded to a multiple of `pad` with
// instance -1.
int2* upload_work(wfp_batch* B, const std::vector<int2>& w, int pad, int& n) {
  std::vector<int2> v = w;
  while (pad > 1 && v.size() % pad) v.push_back(make_int2(-1, 0));
  n = (int)v.size();
  if (v.empty()) return nullptr;
  int2* d = B->alloc<int2>(v.size());
  HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice, B->bs));
  return d;
}

// Work list for a kernel that remaps its blocks to XCDs (xcd_block: XCD k runs
// positions [k * per, (k + 1) * per)).  Each instance's blocks are cut into 8
// contiguous chunks and chunk k goes to XCD k's range, so every XCD gets an
// equal share of every instance (instances differ in cost per block) while
// neighbouring rows, which share sources, stay on one L2.  `ib` holds
// (instance, blocks) pairs; the ranges are padded with instance -1.
std::vector<int2> xcd_balanced(const std::vector<int2>& ib) {
  std::vector<int2> part[8];
  for (const int2& e : ib)
    for (int k = 0; k < 8; ++k)
      for (int b = (int)((int64_t)e.y * k / 8); b < (int)((int64_t)e.y * (k + 1) / 8); ++b)
        part[k].push_back(make_int2(e.x, b));
  size_t per = 0;
  for (int k = 0; k < 8; ++k) per = std::max(per, part[k].size());
  std::vector<int2> out;
  out.reserve(8 * per);
  for (int k = 0; k < 8; ++k) {
    out.insert(out.end(), part[k].begin(), part[k].end());
    out.resize((k + 1) * per, make_int2(-1, 0));
  }
  return out;
}

void build_batch(wfp_batch* B) {
  const int n = (int)B->plans.size();
  std::vector<InstDesc> desc(n);
  // otf, loc4, loc8, g8, g4: (instance, blocks); g8 / g4: instances whose
  // lag blocks are short (the plan's lanes per lag), 4 rows per block
  std::vector<int2> inc, loc4, loc8, wa, wb, wc, dir, til, rows, otf, otfr, g8, g4, rcv, sp, sym, symr;
  for (int i = 0; i < n; ++i) {
    // the spread grid of the separate spread pass
    if (!B->plans[i]->gsp) B->plans[i]->gsp = B->plans[i]->alloc<double>(B->plans[i]->nf);
    const wfp_plan* P = B->plans[i];
    desc[i] = describe(P);
    for (int b = 0; b < (int)nblk(P->nf, 256); ++b) sp.push_back(make_int2(i, b));
    const int M = (int)P->M;
    const int rpb = 256 / desc[i].pp;
    for (int b = 0; b < (int)nblk(M, rpb); ++b) inc.push_back(make_int2(i, b));
    if (P->sym_stored) {
      sym.push_back(make_int2(i, (int)nblk(M, 4)));
      for (int bb = 0; bb < (int)nblk(M, 64); ++bb) symr.push_back(make_int2(i, bb));
    } else if (P->otf) {
      if (P->p != 8) fail(WFP_EDOMAIN, "batched on-the-fly local sums take p = 8");
      otf.push_back(make_int2(i, (int)nblk(M, kOtfRows)));
      for (int bb = 0; bb < (int)nblk(M, 256); ++bb) otfr.push_back(make_int2(i, bb));
      B->lds_otf = std::max(B->lds_otf, (size_t)(P->NQ + kOtfRows) * kOtfChunk * sizeof(double));
    } else if (P->lgrp == 8) {
      g8.push_back(make_int2(i, (int)nblk(M, 4)));
    } else if (P->lgrp == 4) {
      g4.push_back(make_int2(i, (int)nblk(M, 4)));
    } else {
      loc4.push_back(make_int2(i, (int)nblk(M, 4)));
      loc8.push_back(make_int2(i, (int)nblk(M, 8)));
    }
    for (int b = 0; b < P->n1; ++b) wa.push_back(make_int2(i, b));
    for (int b = 0; b < P->n2 / 2 + 1; ++b) wb.push_back(make_int2(i, b));
    for (int b = 0; b < P->n1; ++b) wc.push_back(make_int2(i, b));
    for (int b = 0; b < P->n_direct_tiles; ++b) dir.push_back(make_int2(i, b));
    for (int b = 0; b < P->ntile; ++b) til.push_back(make_int2(i, b));
    for (int b = 0; b < (int)nblk(P->R, 4); ++b) rcv.push_back(make_int2(i, b));   // 4 receivers per block
    if (P->solve_global) {
      for (int b = 0; b < (int)nblk(M, 256); ++b) rows.push_back(make_int2(i, b));
      B->max_sweeps = std::max(B->max_sweeps, P->iters);
    }
    if (P->hist_threads != 256) fail(WFP_EDOMAIN, "batched instances need fine grids of at most 1024 butterflies per row stage");
    B->lds_a = std::max(B->lds_a, (size_t)P->n2 * sizeof(double2));
    B->lds_b = std::max(B->lds_b, 6 * (size_t)P->n1 * sizeof(double2) + 16 * (size_t)P->n1 * sizeof(double4));
    B->lds_til = std::max(B->lds_til, P->lds_jac);
  }
  // sweep lists: global-solve instances by decreasing sweep count
  std::vector<int> order;
  for (int i = 0; i < n; ++i)
    if (B->plans[i]->solve_global && B->plans[i]->iters > 1) order.push_back(i);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return B->plans[a]->iters > B->plans[c]->iters; });
  std::vector<int2> swt, sww;
  B->cnt_swt.assign(std::max(B->max_sweeps, 1), 0);
  B->cnt_sww.assign(std::max(B->max_sweeps, 1), 0);
  for (int i : order) {
    const wfp_plan* P = B->plans[i];
    std::vector<int2>& lst = P->g_wave ? sww : swt;
    const int rpb = P->g_wave ? 4 : 256;
    for (int b = 0; b < (int)nblk(P->M, rpb); ++b) lst.push_back(make_int2(i, b));
    std::vector<int>& cnt = P->g_wave ? B->cnt_sww : B->cnt_swt;
    for (int it = 1; it < P->iters; ++it) cnt[it] = (int)lst.size();
  }
  B->lds_c = B->lds_a;
  B->ends.assign(n, INT64_MAX);
  for (int i = 0; i < n; ++i) desc[i].end = INT64_MAX;
  B->desc_h = desc;
  B->desc_d = B->alloc<InstDesc>(n);
  HIPCHK(hipMemcpyAsync(B->desc_d, desc.data(), n * sizeof(InstDesc), hipMemcpyHostToDevice, B->bs));
  B->wl_inc = upload_work(B, inc, 1, B->n_inc);
  B->wl_loc4 = upload_work(B, xcd_balanced(loc4), 8, B->n_loc4);
  B->wl_loc8 = upload_work(B, xcd_balanced(loc8), 8, B->n_loc8);
  B->wl_a = upload_work(B, wa, 1, B->n_a);
  B->wl_sp = upload_work(B, sp, 1, B->n_sp);
  B->wl_b = upload_work(B, wb, 1, B->n_b);
  B->wl_c = upload_work(B, wc, 1, B->n_c);
  B->wl_dir = upload_work(B, dir, 1, B->n_dir);
  B->wl_til = upload_work(B, til, 1, B->n_til);
  B->wl_rows = upload_work(B, rows, 1, B->n_rows);
  B->wl_otf = upload_work(B, xcd_balanced(otf), 8, B->n_otf);
  B->wl_otfr = upload_work(B, otfr, 1, B->n_otfr);
  B->wl_sym = upload_work(B, xcd_balanced(sym), 8, B->n_sym);
  B->wl_symr = upload_work(B, symr, 1, B->n_symr);
  B->wl_g8 = upload_work(B, xcd_balanced(g8), 8, B->n_g8);
  B->wl_g4 = upload_work(B, xcd_balanced(g4), 8, B->n_g4);
  B->wl_rcv = upload_work(B, rcv, 1, B->n_rcv);
  B->uout_d = B->alloc<double*>(n);
  B->lvl0_d = B->alloc<int64_t>(1);
  HIPCHK(hipMemsetAsync(B->uout_d, 0, n * sizeof(double*), B->bs));
  HIPCHK(hipMemsetAsync(B->lvl0_d, 0, sizeof(int64_t), B->bs));
  B->wl_swt = upload_work(B, swt, 1, B->n_swt);
  B->wl_sww = upload_work(B, sww, 1, B->n_sww);
  if (B->n_otf)
    HIPCHK(hipFuncSetAttribute((const void*)kb_local_otf, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)B->lds_otf));
  B->level_d = B->alloc<int64_t>(1);
  if (B->lds_b > 160 * 1024 || B->lds_til > 160 * 1024) fail(WFP_EDOMAIN, "batched stage needs more than 160 KB of LDS");
  HIPCHK(hipFuncSetAttribute((const void*)kb_hist_b, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipFuncSetAttribute((const void*)kb_solve, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
  HIPCHK(hipStreamSynchronize(B->bs));
}

// The launches of one level (captured into the level's graph): the history
// chain (spread, modes, inverse FFT) and the local sum read only levels before
// L and write disjoint buffers, so the chain is a second branch of the graph
// (on bs2) that joins before the solve.
void enqueue_level(wfp_batch* B) {
  hipStream_t s = B->bs;
  BatchLaunch bl{B->desc_d, nullptr, B->level_d};
  bl.work = B->wl_inc;
  hipLaunchKernelGGL(kb_incident, dim3(B->n_inc), dim3(256), 0, s, bl);
  HIPCHK(hipEventRecord(B->ev_fork, s));
  HIPCHK(hipStreamWaitEvent(B->bs2, B->ev_fork, 0));
  {
    hipStream_t c = B->bs2;
    BatchLaunch bc{B->desc_d, nullptr, B->level_d};
    if (B->spread_pass) {
      bc.work = B->wl_sp;
      hipLaunchKernelGGL(kb_spread_grid, dim3(B->n_sp), dim3(256), 0, c, bc);
    }
    bc.work = B->wl_a;
    hipLaunchKernelGGL(kb_hist_a, dim3(B->n_a), dim3(256), B->lds_a, c, bc, B->spread_pass);
    bc.work = B->wl_b;
    hipLaunchKernelGGL(kb_hist_b, dim3(B->n_b), dim3(512), B->lds_b, c, bc);
    bc.work = B->wl_c;
    hipLaunchKernelGGL(kb_hist_c, dim3(B->n_c), dim3(256), B->lds_c, c, bc);
    HIPCHK(hipEventRecord(B->ev_join, c));
  }
  if (B->loc_rows == 8 && B->n_loc8) {
    bl.work = B->wl_loc8;
    hipLaunchKernelGGL(kb_local, dim3(B->n_loc8), dim3(512), 0, s, bl, B->loc_xcd);
  } else if (B->n_loc4) {
    bl.work = B->wl_loc4;
    hipLaunchKernelGGL(kb_local, dim3(B->n_loc4), dim3(256), 0, s, bl, B->loc_xcd);
  }
  if (B->n_g8) {
    bl.work = B->wl_g8;
    hipLaunchKernelGGL(kb_local_g8, dim3(B->n_g8), dim3(256), 0, s, bl);
  }
  if (B->n_g4) {
    bl.work = B->wl_g4;
    hipLaunchKernelGGL(kb_local_g4, dim3(B->n_g4), dim3(256), 0, s, bl);
  }
  if (B->n_otf) {
    bl.work = B->wl_otf;
    hipLaunchKernelGGL(kb_local_otf, dim3(B->n_otf), dim3(64 * kOtfRows), B->lds_otf, s, bl);
    bl.work = B->wl_otfr;
    hipLaunchKernelGGL(kb_local_otf_reduce, dim3(B->n_otfr), dim3(256), 0, s, bl);
  }
  if (B->n_sym) {
    bl.work = B->wl_sym;
    hipLaunchKernelGGL(kb_local_sym, dim3(B->n_sym), dim3(256), 0, s, bl);
    bl.work = B->wl_symr;
    hipLaunchKernelGGL(kb_local_sym_reduce, dim3(B->n_symr), dim3(64 * kReduceWaves), 0, s, bl);
  }
  HIPCHK(hipStreamWaitEvent(s, B->ev_join, 0));
  if (B->n_dir) {
    bl.work = B->wl_dir;
    hipLaunchKernelGGL(kb_solve_direct, dim3(B->n_dir), dim3(256), 0, s, bl);
  }
  if (B->n_til) {
    bl.work = B->wl_til;
    hipLaunchKernelGGL(kb_solve, dim3(B->n_til), dim3(256), B->lds_til, s, bl);
  }
  if (B->n_rows) {
    bl.work = B->wl_rows;
    hipLaunchKernelGGL(kb_solve_rhs, dim3(B->n_rows), dim3(256), 0, s, bl);
    for (int it = 1; it < B->max_sweeps; ++it) {
      if (B->cnt_swt[it]) {
        bl.work = B->wl_swt;
        hipLaunchKernelGGL(kb_jacobi_sweep, dim3(B->cnt_swt[it]), dim3(256), 0, s, bl, it);
      }
      if (B->cnt_sww[it]) {
        bl.work = B->wl_sww;
        hipLaunchKernelGGL(kb_jacobi_sweep_wave, dim3(B->cnt_sww[it]), dim3(256), 0, s, bl, it);
      }
    }
  }
  if (B->n_rcv) {
    bl.work = B->wl_rcv;
    hipLaunchKernelGGL(kb_receivers, dim3(B->n_rcv), dim3(256), 0, s, bl, B->uout_d, B->lvl0_d);
  }
  hipLaunchKernelGGL(kb_advance, dim3(1), dim3(64), 0, s, B->level_d);
}

// Receiver outputs for the next run (NULL: none).  The captured level reads
// the pointers and the start level from device memory, so they are written
// here after the batch's earlier work has finished with them.
void set_outputs(wfp_batch* B, double* const* u_recv_out) {
  if (!B->n_rcv || (!u_recv_out && !B->uout_set)) return;
  HIPCHK(hipStreamSynchronize(B->bs));
  const size_t n = B->plans.size();
  std::vector<double*> h(n, nullptr);
  if (u_recv_out)
    for (size_t i = 0; i < n; ++i) h[i] = u_recv_out[i];
  HIPCHK(hipMemcpy(B->uout_d, h.data(), n * sizeof(double*), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(B->lvl0_d, &B->level, sizeof(int64_t), hipMemcpyHostToDevice));
  B->uout_set = u_recv_out != nullptr;
}

void drop_graph(wfp_batch* B) {
  if (B->exec) HIPCHK(hipGraphExecDestroy(B->exec));
  if (B->graph) HIPCHK(hipGraphDestroy(B->graph));
  B->exec = nullptr;
  B->graph = nullptr;
}

void capture(wfp_batch* B) {
  if (B->exec) return;
  HIPCHK(hipStreamBeginCapture(B->bs, hipStreamCaptureModeThreadLocal));
  enqueue_level(B);
  HIPCHK(hipStreamEndCapture(B->bs, &B->graph));
  HIPCHK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
}

// Each instance's own level: the batch level, or its end once reached.
void sync_plan_levels(wfp_batch* B) {
  for (size_t i = 0; i < B->plans.size(); ++i) B->plans[i]->level = std::min(B->level, B->ends[i]);
}

void set_level(wfp_batch* B, int64_t L) {
  B->level = L;
  HIPCHK(hipMemcpyAsync(B->level_d, &B->level, sizeof(int64_t), hipMemcpyHostToDevice, B->bs));
  HIPCHK(hipStreamSynchronize(B->bs));
  sync_plan_levels(B);
}

void run_batch(wfp_batch* B, int64_t n) {
  capture(B);
  for (int64_t i = 0; i < n; ++i) HIPCHK(hipGraphLaunch(B->exec, B->bs));
  B->level += n;
  sync_plan_levels(B);
}

void reset_batch(wfp_batch* B) {
  for (wfp_plan* P : B->plans)
    if (wfp_reset(P) != WFP_OK) fail(WFP_EHIP, g_last_error);
  HIPCHK(hipStreamSynchronize(B->bs));
  set_level(B, 0);
}

// Number of ordered (target, source) pairs closer than delta (periodic box).
int64_t count_pairs(const double* x, int64_t M, double delta) {
  std::vector<double> xs(x, x + M);
  std::sort(xs.begin(), xs.end());
  // sources within delta of each target, by two pointers over three copies of
  // the circle (targets in the middle one)
  std::vector<double> ext(3 * M);
  for (int64_t i = 0; i < M; ++i) {
    ext[i] = xs[i] - kTwoPi;
    ext[i + M] = xs[i];
    ext[i + 2 * M] = xs[i] + kTwoPi;
  }
  int64_t tot = 0, hi = M, lo = 0;
  for (int64_t j = M; j < 2 * M; ++j) {
    while (hi < 3 * M && ext[hi] - ext[j] < delta) ++hi;
    while (ext[j] - ext[lo] >= delta) ++lo;
    tot += std::min<int64_t>(hi - lo, M);
  }
  return tot;
}

// Local-weight mode of every instance whose parameters leave it to the
// library: stored weights for the instances with the fewest pairs while their
// packed weights fit in 45 % of the free device memory (and the set-up array
// of one instance in 25 %), on the fly for the rest.
std::vector<int> choose_local_modes(int n, const wfp_problem* probs, const wfp_params* pars) {
  size_t fr = 0, to = 0;
  HIPCHK(hipMemGetInfo(&fr, &to));
  std::vector<int> mode(n);
  std::vector<std::pair<double, int>> cand;
  std::vector<double> packed(n), dense(n);
  std::vector<char> many(n, 0);
  for (int i = 0; i < n; ++i) {
    mode[i] = pars[i].local_mode;
    if (mode[i] != 0) continue;
    const double eps = pars[i].eps_window > 0 ? pars[i].eps_window : 1e-12;
    const double gamma = pars[i].gamma > 0 ? pars[i].gamma : 0.5;
    const int W = pars[i].W > 0 ? pars[i].W : (int)std::lround(2.0 * std::log(1.0 / eps) / (kPi * gamma));
    const int p = pars[i].p > 0 ? pars[i].p : 8;
    const double pairs = (double)count_pairs(probs[i].x, probs[i].M, W * pars[i].dt);
    packed[i] = 8.0 * pairs * (W / 2 + p);        // nonzero lags per pair
    dense[i] = 8.0 * pairs * (W + p / 2);
    many[i] = pairs >= kPairOnceNeighbours * (double)probs[i].M ? 1 : 0;
    cand.push_back({packed[i], i});
  }
  std::sort(cand.begin(), cand.end());
  double used = 0.0;
  for (auto& c : cand) {
    const int i = c.second;
    // as for a plan: once per unordered pair (half the bytes) for springs
    // with many neighbours or where per-pair weights would not fit
    const bool fits1 = used + packed[i] <= 0.45 * (double)fr && dense[i] <= 0.25 * (double)fr;
    const bool fits3 = used + 0.5 * packed[i] <= 0.45 * (double)fr && 0.5 * dense[i] <= 0.25 * (double)fr;
    if (fits3 && (many[i] || !fits1)) {
      mode[i] = 3;
      used += 0.5 * packed[i];
    } else if (fits1) {
      mode[i] = 1;
      used += packed[i];
    } else {
      mode[i] = 2;
    }
  }
  return mode;
}

}  // namespace

extern "C" {

wfp_status wfp_batch_create(int32_t n, const wfp_problem* probs, const wfp_params* pars, void* stream,
                            wfp_batch** out) {
  if (!out || n < 1 || !probs || !pars) {
    g_last_error = "batch needs n >= 1, problems, parameters and an output handle";
    return WFP_EINVAL;
  }
  *out = nullptr;
  for (int32_t i = 0; i < n; ++i) {
    if (probs[i].boundary != WFP_PERIODIC) {
      g_last_error = "the batched form covers periodic problems";
      return WFP_EDOMAIN;
    }
    if (pars[i].checkpoint_every != 0) {
      // its levels are marched by the batch's own launches, which neither
      // store checkpoints nor record levels for a gradient pass
      g_last_error = "the batched form takes checkpoint_every 0";
      return WFP_EINVAL;
    }
  }
  wfp_batch* B = new wfp_batch();
  wfp_status st = guard([&] {
    HIPCHK(hipGetDevice(&B->device));
    B->user_stream = (hipStream_t)stream;
    HIPCHK(hipStreamCreateWithFlags(&B->bs, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&B->bs2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
    const std::vector<int> modes = choose_local_modes(n, probs, pars);
    for (int32_t i = 0; i < n; ++i) {
      wfp_plan* P = nullptr;
      // the batch overlaps instances instead of streams: one stream per plan
      wfp_params pi = pars[i];
      pi.overlap_cus = -1;
      pi.local_mode = modes[i];
      const wfp_status s = wfp_plan_create(&probs[i], &pi, B->bs, &P);
      if (s != WFP_OK) throw Error{s, "instance " + std::to_string(i) + ": " + g_last_error};
      B->plans.push_back(P);
    }
    build_batch(B);
    set_level(B, 0);
  });
  if (st != WFP_OK) {
    delete B;
    return st;
  }
  *out = B;
  return WFP_OK;
}

void wfp_batch_destroy(wfp_batch* B) {
  if (!B) return;
  (void)hipStreamSynchronize(B->bs);
  delete B;
}

wfp_status wfp_batch_run(wfp_batch* B, int64_t n_steps, double* const* u_recv_out, double* const* sigma_final) {
  if (!B || n_steps < 0) {
    g_last_error = "bad batch or step count";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(B->device));
    set_outputs(B, u_recv_out);
    HIPCHK(hipEventRecord(B->ev_in, B->user_stream));
    HIPCHK(hipStreamWaitEvent(B->bs, B->ev_in, 0));
    run_batch(B, n_steps);
    if (sigma_final && B->level > 0) {
      for (size_t i = 0; i < B->plans.size(); ++i) {
        const wfp_plan* P = B->plans[i];
        if (!sigma_final[i] || P->level < 1) continue;
        // the instance's own last level (its end level, once reached)
        const double* last = P->hist + (int64_t)(((P->level - 1) % P->NH + P->NH) % P->NH) * P->M;
        hipLaunchKernelGGL(k_unsort, dim3(nblk(P->M, 256)), dim3(256), 0, B->bs, (int)P->M, P->perm, last,
                           sigma_final[i]);
      }
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipEventRecord(B->ev_out, B->bs));
    HIPCHK(hipStreamWaitEvent(B->user_stream, B->ev_out, 0));
  });
}

wfp_status wfp_batch_set_levels(wfp_batch* B, const int64_t* n_levels) {
  if (!B) {
    g_last_error = "NULL batch";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(B->device));
    const size_t n = B->plans.size();
    // the captured levels read the table: earlier replays finish first
    HIPCHK(hipStreamSynchronize(B->bs));
    for (size_t i = 0; i < n; ++i) {
      const int64_t e = (n_levels && n_levels[i] > 0) ? n_levels[i] : INT64_MAX;
      B->ends[i] = e;
      B->desc_h[i].end = e;
    }
    HIPCHK(hipMemcpy(B->desc_d, B->desc_h.data(), n * sizeof(InstDesc), hipMemcpyHostToDevice));
    sync_plan_levels(B);
  });
}

wfp_status wfp_batch_reset(wfp_batch* B) {
  if (!B) {
    g_last_error = "NULL batch";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(B->device));
    HIPCHK(hipEventRecord(B->ev_in, B->user_stream));
    HIPCHK(hipStreamWaitEvent(B->bs, B->ev_in, 0));
    reset_batch(B);
  });
}

wfp_status wfp_batch_autotune(wfp_batch* B, int32_t trial_levels, int32_t* rows_per_block, int32_t* xcd_remap,
                              int32_t* spread_pass) {
  if (!B || trial_levels < 1) {
    g_last_error = "autotune needs a batch and trial_levels >= 1";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(B->device));
    if (B->level != 0) fail(WFP_ESTATE, "autotune runs from level 0 (call wfp_batch_reset first)");
    set_outputs(B, nullptr);   // trial levels write no receiver rows
    HIPCHK(hipStreamSynchronize(B->user_stream));
    hipEvent_t a, c;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&c));
    float best = 1e30f;
    int br = 4, bx = 1, bs = 0;
    // (rows per block, XCD remap, spread tile)
    const int cand[8][3] = {{4, 1, 0}, {8, 1, 0}, {4, 0, 0}, {8, 0, 0},
                            {4, 1, 1}, {8, 1, 1}, {4, 0, 1}, {8, 0, 1}};
    for (const auto& cd : cand) {
      B->loc_rows = cd[0];
      B->loc_xcd = cd[1];
      B->spread_pass = cd[2];
      drop_graph(B);
      capture(B);
      HIPCHK(hipGraphLaunch(B->exec, B->bs));       // warm-up level
      HIPCHK(hipEventRecord(a, B->bs));
      for (int32_t i = 0; i < trial_levels; ++i) HIPCHK(hipGraphLaunch(B->exec, B->bs));
      HIPCHK(hipEventRecord(c, B->bs));
      HIPCHK(hipEventSynchronize(c));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, a, c));
      if (ms < best) {
        best = ms;
        br = cd[0];
        bx = cd[1];
        bs = cd[2];
      }
      reset_batch(B);
    }
    HIPCHK(hipEventDestroy(a));
    HIPCHK(hipEventDestroy(c));
    B->loc_rows = br;
    B->loc_xcd = bx;
    B->spread_pass = bs;
    drop_graph(B);
    if (rows_per_block) *rows_per_block = br;
    if (xcd_remap) *xcd_remap = bx;
    if (spread_pass) *spread_pass = bs;
  });
}

wfp_status wfp_batch_set_shape(wfp_batch* B, int32_t rows_per_block, int32_t xcd_remap, int32_t spread_pass) {
  if (!B || (rows_per_block != 4 && rows_per_block != 8) || (xcd_remap != 0 && xcd_remap != 1) ||
      (spread_pass != 0 && spread_pass != 1)) {
    g_last_error = "set_shape takes a batch, rows_per_block 4 or 8, xcd_remap 0 or 1, spread_pass 0 or 1";
    return WFP_EINVAL;
  }
  return guard([&] {
    HIPCHK(hipSetDevice(B->device));
    // the captured level is rebuilt at the next run, after the earlier levels
    HIPCHK(hipStreamSynchronize(B->bs));
    B->loc_rows = rows_per_block;
    B->loc_xcd = xcd_remap;
    B->spread_pass = spread_pass;
    drop_graph(B);
  });
}

wfp_status wfp_batch_size(const wfp_batch* B, int32_t* n, int64_t* level) {
  if (!B) {
    g_last_error = "NULL batch";
    return WFP_EINVAL;
  }
  if (n) *n = (int32_t)B->plans.size();
  if (level) *level = B->level;
  return WFP_OK;
}

wfp_plan* wfp_batch_plan(wfp_batch* B, int32_t i) {
  if (!B || i < 0 || i >= (int32_t)B->plans.size()) {
    g_last_error = "bad batch or instance index";
    return nullptr;
  }
  return B->plans[i];
}

}  // extern "C"
