// C ABI of the bbFMM library (include/bbfmm.h): argument validation, object lifetimes,
// host precompute and upload, and the stream-ordered pass sequence of an apply.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "internal.h"

namespace bbfmm {

static thread_local std::string g_last_error;

void set_error(bbfmm_status code, const std::string& msg) {
  (void)code;
  g_last_error = msg;
}

bbfmm_status fail(bbfmm_status code, const std::string& msg) {
  set_error(code, msg);
  return code;
}

namespace {

template <typename T>
hipError_t dmalloc(T** p, size_t count, long long* bytes) {
  *p = nullptr;
  if (count == 0) return hipSuccess;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e == hipSuccess && bytes) *bytes += (long long)(count * sizeof(T));
  return e;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

PassGeom geom_of(const bbfmm_plan* pl) {
  const bbfmm_tree* t = pl->tree;
  PassGeom g;
  g.xs = t->xs; g.ys = t->ys; g.zs = t->zs;
  g.perm = t->perm; g.leaf_of = t->leaf_of; g.leaf_start = t->leaf_start;
  g.n = t->n; g.depth = t->depth;
  for (int r = 0; r < 3; ++r) g.lo[r] = t->lo[r];
  g.width = t->width;
  g.tk = pl->d_tk; g.m2m = pl->d_m2m; g.h_m2m = pl->h_m2m.data();
  g.order = pl->order; g.kernel = pl->kernel; g.c = pl->c;
  return g;
}

bool valid_kernel(int k) {
  return k == kInvR || k == kInvSqrtR2C2 || k == kHelmCos || k == kHelmSin || k == kR2 || k == kR4;
}

// Compressed factors of representative p's operator K (row-major l^3 x l^3) by the chosen
// compressor; returns the rank.
int compress_operator(const double* K, int order, int p, double eps, int compressor, std::vector<double>& uf,
                      std::vector<double>& vf) {
  const int nn = order * order * order;
  if (compressor == BBFMM_COMPRESS_SVD) return compress_svd(K, nn, eps, uf, vf);
  // Q with K_p^T = K_p[Q][:, Q]: the permutation of -t_p
  const auto& t = representatives()[p];
  const int mt[3] = {-t[0], -t[1], -t[2]};
  std::vector<int32_t> q(nn);
  sigma_table(order, symmetry_of(mt).perm_id, q.data());
  return compress_aca(K, nn, q.data(), eps, uf, vf);
}

void free_buffers(bbfmm_plan* p) {
  dfree(p->W); p->W = nullptr;
  for (int s = 0; s < 2; ++s) {
    dfree(p->F[s]); p->F[s] = nullptr;
    dfree(p->qs[s]); p->qs[s] = nullptr;
    p->slot_nrhs[s] = 0;
  }
  dfree(p->phis); p->phis = nullptr;
  dfree(p->d_what); p->d_what = nullptr;
  dfree(p->d_fhat); p->d_fhat = nullptr;
  p->nrhs_cap = 0;
  p->buffer_bytes = 0;
}

bbfmm_status ensure_buffers(bbfmm_plan* p, int nrhs, int slot) {
  const bbfmm_tree* t = p->tree;
  if (nrhs > p->nrhs_cap) {
    free_buffers(p);
    long long bytes = 0;
    if (t->depth >= 2) {
      BBFMM_HIP_TRY(dmalloc(&p->W, (size_t)p->exp_elems * nrhs, &bytes));
      BBFMM_HIP_TRY(dmalloc(&p->F[0], (size_t)p->exp_elems * nrhs, &bytes));
      BBFMM_HIP_TRY(dmalloc(&p->phis, (size_t)t->n * nrhs, &bytes));
      if (p->variant != 0) {
        // What / Fhat of every M2L level side by side
        const int rp = *std::max_element(p->sa_rp.begin(), p->sa_rp.end());
        size_t cells = 0;
        for (int l = 2; l <= t->depth; ++l) cells += (size_t)1 << (3 * l);
        const size_t elems = cells * rp * nrhs;
        BBFMM_HIP_TRY(dmalloc(&p->d_what, elems, &bytes));
        BBFMM_HIP_TRY(dmalloc(&p->d_fhat, elems, &bytes));
      }
    }
    BBFMM_HIP_TRY(dmalloc(&p->qs[0], (size_t)t->n * nrhs, &bytes));
    p->nrhs_cap = nrhs;
    p->buffer_bytes = bytes;
  }
  if (slot == 1 && p->qs[1] == nullptr) {
    long long bytes = 0;
    if (t->depth >= 2) BBFMM_HIP_TRY(dmalloc(&p->F[1], (size_t)p->exp_elems * p->nrhs_cap, &bytes));
    BBFMM_HIP_TRY(dmalloc(&p->qs[1], (size_t)t->n * p->nrhs_cap, &bytes));
    p->buffer_bytes += bytes;
  }
  return BBFMM_OK;
}

// SA / SArcmp M2L of levels 2..depth (only_level < 0, W and F the whole expansion arrays) or of
// one level (W and F that level's arrays). Each level gets its own What / Fhat region.
bbfmm_status sa_levels(const bbfmm_plan* p, int nrhs, const double* W, double* F, int only_level, hipStream_t s) {
  SALevelArgs lv[kSAMaxLevels];
  int nlev = 0;
  const int rp_max = *std::max_element(p->sa_rp.begin(), p->sa_rp.end());
  long long cell_off = 0;
  for (int l = 2; l <= p->tree->depth; ++l) {
    const long long cells = 1LL << (3 * l);
    if (only_level >= 0 && l != only_level) {
      cell_off += cells;
      continue;
    }
    if (nlev == kSAMaxLevels) return fail(BBFMM_EUNSUPPORTED, "too many SA levels");
    const int set = p->set_of_level[l];
    SALevelArgs& a = lv[nlev++];
    std::memset(&a, 0, sizeof(a));
    a.W = only_level >= 0 ? W : W + p->level_off[l] * nrhs;
    a.F = only_level >= 0 ? F : F + p->level_off[l] * nrhs;
    a.what = p->d_what + cell_off * rp_max * nrhs;
    a.fhat = p->d_fhat + cell_off * rp_max * nrhs;
    a.u = p->d_sa + p->sa_u_off[set];
    a.ut = p->d_sa + p->sa_ut_off[set];
    a.ops = p->d_sa;
    a.off = p->d_sa_off + (size_t)set * 512;
    a.rank = p->d_sa_rank + (size_t)set * 512;
    a.tab = p->d_tab;
    a.level = l; a.n = p->nn; a.r = p->sa_r[set]; a.rp = p->sa_rp[set]; a.nrhs = nrhs;
    a.max_op_doubles = p->sa_max_op[set];
    a.stage_ops = p->variant == BBFMM_VARIANT_SA ? 1 : 0;
    a.scale = p->scale_of_level[l];
    cell_off += cells;
  }
  if (nlev == 0) return BBFMM_OK;
  BBFMM_HIP_TRY(launch_sa_levels(lv, nlev, s));
  return BBFMM_OK;
}

M2LArgs m2l_args(const bbfmm_plan* p, int nrhs, const double* W, double* F, int only_level) {
  const bbfmm_tree* t = p->tree;
  M2LArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nrhs = nrhs;
  int k = 0;
  for (int l = t->depth; l >= 2; --l) {
    if (only_level >= 0 && l != only_level) continue;
    M2LLevel& lv = a.lv[k++];
    lv.W = only_level >= 0 ? W : W + p->level_off[l] * nrhs;
    lv.F = only_level >= 0 ? F : F + p->level_off[l] * nrhs;
    lv.level = l;
    lv.side = 1 << l;
    lv.npar = 1 << (3 * (l - 1));
    lv.set = p->set_of_level[l];
    lv.scale = p->scale_of_level[l];
  }
  a.nlev = k;
  a.ops_hi = p->ops_hi; a.ops_lo = p->ops_lo;
  a.op_off = p->d_op_off; a.op_rank = p->d_op_rank;
  a.max_rank = p->lowrank ? *std::max_element(p->ranks.begin(), p->ranks.end()) : 0;
  a.tab = p->d_tab; a.grp = p->d_grp; a.sig = p->d_sig; a.siginv = p->d_siginv;
  a.zeros = p->d_zeros;
  // the split of the last round needs the whole-apply launch (all levels)
  if (only_level < 0) {
    a.scratch = p->d_split;
    a.split_cap = p->split_cap;
    a.tcount = p->d_tcount;
    a.tcount_len = p->tcount_len;
  }
  return a;
}

AdaptiveGeom ageom_of(const bbfmm_plan* pl) {
  const bbfmm_tree* t = pl->tree;
  AdaptiveGeom g;
  g.xs = t->xs; g.ys = t->ys; g.zs = t->zs;
  g.perm = t->perm; g.leaf_of = t->leaf_of;
  g.n = t->n;
  g.start = t->d_start; g.end = t->d_end; g.cen = t->d_cen;
  g.child_begin = t->d_child_begin; g.child_end = t->d_child_end; g.oct = t->d_oct;
  g.tk = pl->d_tk; g.m2m = pl->d_m2m; g.h_m2m = pl->h_m2m.data();
  g.order = pl->order; g.kernel = pl->kernel; g.c = pl->c;
  return g;
}

void free_tree_arrays(bbfmm_tree* t) {
  dfree(t->xs); dfree(t->ys); dfree(t->zs); dfree(t->perm); dfree(t->leaf_of); dfree(t->leaf_start);
  dfree(t->d_start); dfree(t->d_end); dfree(t->d_cen); dfree(t->d_child_begin); dfree(t->d_child_end);
  dfree(t->d_oct); dfree(t->d_leaves); dfree(t->d_leaf_pos); dfree(t->d_u_off); dfree(t->d_u_idx);
  dfree(t->d_w_off); dfree(t->d_w_idx); dfree(t->d_x_node); dfree(t->d_x_off); dfree(t->d_x_idx);
  dfree(t->d_m2l_tgt); dfree(t->d_vsrc); dfree(t->d_move_flag);
  t->d_move_flag = nullptr;
  t->xs = t->ys = t->zs = nullptr;
  t->perm = t->leaf_of = t->leaf_start = nullptr;
}

// Tiles the adaptive M2L segments for `nrhs` and uploads them (waits for the stream first: an
// M2L still running may read the previous tiling).
bbfmm_status adaptive_segments(bbfmm_plan* p, int nrhs, hipStream_t s) {
  if (p->segs_nrhs == nrhs || p->h_segs.empty()) return BBFMM_OK;
  BBFMM_HIP_TRY(hipStreamSynchronize(s));
  const int cols = m2l_block_cols(p->lowrank, p->order, p->prec);
  long long blocks = 0;
  for (M2LLevel& sg : p->h_segs) {
    const long long c = (long long)sg.npar * nrhs;
    sg.ntiles = (int)((c + cols - 1) / cols);
    sg.block_begin = (int)blocks;
    blocks += sg.ntiles;
  }
  if (blocks > 0x7fffff00LL) return fail(BBFMM_EUNSUPPORTED, "too many M2L blocks");
  BBFMM_HIP_TRY(hipMemcpy(p->d_segs, p->h_segs.data(), p->h_segs.size() * sizeof(M2LLevel),
                          hipMemcpyHostToDevice));
  p->seg_blocks = (int)blocks;
  p->segs_nrhs = nrhs;
  return BBFMM_OK;
}

M2LArgs adaptive_m2l_args(const bbfmm_plan* p, int nrhs, const double* W, double* F) {
  const bbfmm_tree* t = p->tree;
  M2LArgs a;
  std::memset(&a, 0, sizeof(a));
  a.nrhs = nrhs;
  a.lv[0].W = W;
  a.lv[0].F = F;
  a.nlev = 0;
  a.nblocks = p->seg_blocks;
  a.cols = m2l_block_cols(p->lowrank, p->order, p->prec);
  a.ops_hi = p->ops_hi; a.ops_lo = p->ops_lo;
  a.op_off = p->d_op_off; a.op_rank = p->d_op_rank;
  a.max_rank = p->lowrank ? *std::max_element(p->ranks.begin(), p->ranks.end()) : 0;
  a.tab = p->d_tab; a.grp = p->d_grp; a.sig = p->d_sig; a.siginv = p->d_siginv;
  a.zeros = p->d_zeros;
  a.segs = p->d_segs;
  a.nsegs = (int)p->h_segs.size();
  a.tgt = p->m2l_tgt;
  a.vsrc = p->m2l_vsrc;
  (void)t;
  return a;
}

enum Pass { kPassStart = -1, kGather = 0, kP2M, kM2M, kM2L, kL2L, kL2P, kP2P, kNumPasses };

// Records an event tagged with the pass that just ended (tracing only).
hipError_t mark(bbfmm_plan* p, const Work& wk, int tag, hipStream_t s) {
  if (!p->timing || !wk.trace) return hipSuccess;
  if (p->ev_used == p->ev_pool.size()) {
    hipEvent_t e;
    hipError_t er = hipEventCreate(&e);
    if (er != hipSuccess) return er;
    p->ev_pool.push_back(e);
    p->ev_tag.push_back(0);
  }
  p->ev_tag[p->ev_used] = tag;
  return hipEventRecord(p->ev_pool[p->ev_used++], s);
}

// The chain on an adaptive tree: P2M at the leaves, M2M up to level 2, M2L over the V lists,
// P2L over the X lists, L2L down, L2P and M2P over the W lists at the leaves, and the near field
// over the U lists. P2L is timed with L2L and M2P with L2P.
bbfmm_status run_chain_adaptive(bbfmm_plan* p, const double* in, int nrhs, double* out, const Work& wk,
                                hipStream_t s) {
  const bbfmm_tree* t = p->tree;
  const AdaptiveTopology& T = t->topo;
  const AdaptiveGeom g = ageom_of(p);
  double* qs = wk.qs;
  BBFMM_HIP_TRY(mark(p, wk, kPassStart, s));
  BBFMM_HIP_TRY(launch_gather_rows(in, t->perm, t->n, nrhs, qs, s));
  BBFMM_HIP_TRY(mark(p, wk, kGather, s));
  const double* far = nullptr;
  const int nleaves = (int)T.leaves.size();
  if (t->depth >= 2) {
    bbfmm_status st = adaptive_segments(p, nrhs, s);
    if (st != BBFMM_OK) return st;
    double* W = wk.W;
    double* F = wk.F;
    BBFMM_HIP_TRY(launch_ad_p2m(g, t->d_leaves, nleaves, qs, nrhs, W, s));
    BBFMM_HIP_TRY(mark(p, wk, kP2M, s));
    for (int l = t->depth - 1; l >= 2; --l)
      BBFMM_HIP_TRY(launch_ad_m2m(g, T.level_off[l], T.level_off[l + 1], W, nrhs, s));
    BBFMM_HIP_TRY(mark(p, wk, kM2M, s));
    BBFMM_HIP_TRY(launch_fill_zero(F, p->exp_elems * nrhs, s));
    const M2LArgs a = adaptive_m2l_args(p, nrhs, W, F);
    BBFMM_HIP_TRY(launch_m2l(p->order, p->lowrank, p->prec, a, s));
    BBFMM_HIP_TRY(mark(p, wk, kM2L, s));
    BBFMM_HIP_TRY(launch_ad_p2l(g, t->d_x_node, t->d_x_off, t->d_x_idx, (int)T.x_node.size(), qs, nrhs, F, s));
    for (int l = 2; l < t->depth; ++l)
      BBFMM_HIP_TRY(launch_ad_l2l(g, T.level_off[l], T.level_off[l + 1], F, nrhs, s));
    BBFMM_HIP_TRY(mark(p, wk, kL2L, s));
    BBFMM_HIP_TRY(launch_ad_l2p(g, t->d_leaves, nleaves, F, nrhs, wk.phis, s));
    if (!T.w_idx.empty())
      BBFMM_HIP_TRY(launch_ad_m2p(g, t->d_leaves, t->d_w_off, t->d_w_idx, nleaves, W, nrhs, wk.phis, s));
    BBFMM_HIP_TRY(mark(p, wk, kL2P, s));
    far = wk.phis;
  }
  BBFMM_HIP_TRY(launch_ad_p2p_scatter(g, t->d_leaf_pos, t->d_u_off, t->d_u_idx, qs, far, nrhs, out, s));
  BBFMM_HIP_TRY(mark(p, wk, kP2P, s));
  return BBFMM_OK;
}

// One forward pass of the chain on `in` (caller order) into `out` (caller order) with the work
// arrays `wk`.
bbfmm_status run_chain_in(bbfmm_plan* p, const double* in, int nrhs, double* out, const Work& wk, hipStream_t s) {
  const bbfmm_tree* t = p->tree;
  if (t->adaptive) return run_chain_adaptive(p, in, nrhs, out, wk, s);
  const PassGeom g = geom_of(p);
  double* qs = wk.qs;
  BBFMM_HIP_TRY(mark(p, wk, kPassStart, s));
  BBFMM_HIP_TRY(launch_gather_rows(in, t->perm, t->n, nrhs, qs, s));
  BBFMM_HIP_TRY(mark(p, wk, kGather, s));
  const double* far = nullptr;
  if (t->depth >= 2) {
    double* W = wk.W;
    double* F = wk.F;
    const int d = t->depth;
    BBFMM_HIP_TRY(launch_p2m(g, qs, nrhs, W + p->level_off[d] * nrhs, s));
    BBFMM_HIP_TRY(mark(p, wk, kP2M, s));
    for (int l = d - 1; l >= 2; --l)
      BBFMM_HIP_TRY(launch_m2m(g, l, W + p->level_off[l + 1] * nrhs, W + p->level_off[l] * nrhs, nrhs, s));
    BBFMM_HIP_TRY(mark(p, wk, kM2M, s));
    if (p->variant != 0) {
      const bbfmm_status st2 = sa_levels(p, nrhs, W, F, -1, s);
      if (st2 != BBFMM_OK) return st2;
    } else if (p->sparse_m2l) {
      // only targets holding points are computed: the locals of empty cells start at zero
      bbfmm_status st2 = adaptive_segments(p, nrhs, s);
      if (st2 != BBFMM_OK) return st2;
      BBFMM_HIP_TRY(launch_fill_zero(F, p->exp_elems * nrhs, s));
      const M2LArgs a = adaptive_m2l_args(p, nrhs, W, F);
      BBFMM_HIP_TRY(launch_m2l(p->order, p->lowrank, p->prec, a, s));
    } else {
      const M2LArgs a = m2l_args(p, nrhs, W, F, -1);
      BBFMM_HIP_TRY(launch_m2l(p->order, p->lowrank, p->prec, a, s));
    }
    BBFMM_HIP_TRY(mark(p, wk, kM2L, s));
    for (int l = 3; l <= d; ++l)
      BBFMM_HIP_TRY(launch_l2l(g, l - 1, F + p->level_off[l - 1] * nrhs, F + p->level_off[l] * nrhs, nrhs, s));
    BBFMM_HIP_TRY(mark(p, wk, kL2L, s));
    BBFMM_HIP_TRY(launch_l2p(g, F + p->level_off[d] * nrhs, nrhs, wk.phis, s));
    BBFMM_HIP_TRY(mark(p, wk, kL2P, s));
    far = wk.phis;
  }
  BBFMM_HIP_TRY(launch_p2p_scatter(g, qs, far, nrhs, out, s));
  BBFMM_HIP_TRY(mark(p, wk, kP2P, s));
  return BBFMM_OK;
}

// The chain with the plan's own buffers: slot 0 keeps the locals of an apply, slot 1 those of an
// adjoint apply (for bbfmm_eval_grad).
bbfmm_status run_chain(bbfmm_plan* p, const double* in, int nrhs, double* out, int slot, hipStream_t s) {
  bbfmm_status st = ensure_buffers(p, nrhs, slot);
  if (st != BBFMM_OK) return st;
  const Work wk{p->qs[slot], p->W, p->F[slot], p->phis, true};
  st = run_chain_in(p, in, nrhs, out, wk, s);
  if (st == BBFMM_OK) p->slot_nrhs[slot] = nrhs;
  return st;
}

std::vector<int> octant_tables(std::vector<int>* grp) {
  std::vector<int> tab(8 * kFarPerOctant);
  grp->assign(8 * 17, 0);
  for (int o = 0; o < 8; ++o) octant_table(o, &tab[o * kFarPerOctant], &(*grp)[o * 17]);
  return tab;
}

// Root cube from the points' bounding box: the given cube (every point inside) or the tight
// bounding cube enlarged by 1e-12 relative, centred on the box.
bbfmm_status root_of(const double bblo[3], const double bbhi[3], const double root_lo[3], double root_width,
                     bbfmm_tree* t) {
  if (root_width > 0) {
    for (int r = 0; r < 3; ++r) {
      t->lo[r] = root_lo[r];
      if (bblo[r] < root_lo[r] || bbhi[r] > root_lo[r] + root_width)
        return fail(BBFMM_EINVAL, "a point lies outside the root cube");
    }
    t->width = root_width;
  } else {
    double ext = 0.0;
    for (int r = 0; r < 3; ++r) ext = std::max(ext, bbhi[r] - bblo[r]);
    if (!(ext > 0.0)) ext = 1.0;
    const double w = ext * (1.0 + 1e-12);
    for (int r = 0; r < 3; ++r) t->lo[r] = bblo[r] - 0.5 * (w - (bbhi[r] - bblo[r]));
    t->width = w;
  }
  return BBFMM_OK;
}

// Uploads the host topology of an adaptive tree.
hipError_t upload_topology(bbfmm_tree* t, long long* bytes) {
  const AdaptiveTopology& T = t->topo;
  const int nn = T.level_off.empty() ? 0 : T.level_off.back();
  std::vector<double> cen(4 * (size_t)nn);
  std::vector<unsigned char> oct(nn);
  for (int g = 0; g < nn; ++g) {
    for (int r = 0; r < 3; ++r) cen[4 * (size_t)g + r] = T.center[3 * (size_t)g + r];
    cen[4 * (size_t)g + 3] = T.half[g];
    oct[g] = (unsigned char)(T.key[g] & 7);
  }
  auto up = [&](auto** dst, const auto& v) -> hipError_t {
    using E = typename std::remove_reference<decltype(v)>::type::value_type;
    hipError_t e = dmalloc(dst, v.size(), bytes);
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpy(*dst, v.data(), v.size() * sizeof(E), hipMemcpyHostToDevice);
  };
  hipError_t e = up(&t->d_start, T.start);
  if (e == hipSuccess) e = up(&t->d_end, T.end);
  if (e == hipSuccess) e = up(&t->d_cen, cen);
  if (e == hipSuccess) e = up(&t->d_child_begin, T.child_begin);
  if (e == hipSuccess) e = up(&t->d_child_end, T.child_end);
  if (e == hipSuccess) e = up(&t->d_oct, oct);
  if (e == hipSuccess) e = up(&t->d_leaves, T.leaves);
  if (e == hipSuccess) e = up(&t->d_leaf_pos, T.leaf_pos);
  if (e == hipSuccess) e = up(&t->d_u_off, T.u_off);
  if (e == hipSuccess) e = up(&t->d_u_idx, T.u_idx);
  if (e == hipSuccess) e = up(&t->d_w_off, T.w_off);
  if (e == hipSuccess) e = up(&t->d_w_idx, T.w_idx);
  if (e == hipSuccess) e = up(&t->d_x_node, T.x_node);
  if (e == hipSuccess) e = up(&t->d_x_off, T.x_off);
  if (e == hipSuccess) e = up(&t->d_x_idx, T.x_idx);
  if (e == hipSuccess) e = up(&t->d_m2l_tgt, T.m2l_tgt);
  if (e == hipSuccess) e = up(&t->d_vsrc, T.vsrc);
  return e;
}

// Segments of the full-rank M2L on a uniform tree restricted to cells that hold points: per
// (level, octant) the non-empty target cells in Morton order, and their source lists (empty or
// outside sources are absent, so blocks skip transfer vectors none of their targets needs).
bbfmm_status build_sparse_uniform(bbfmm_plan* p, hipStream_t s, long long* bytes) {
  const bbfmm_tree* t = p->tree;
  const int d = t->depth, nn = p->nn;
  std::vector<int> ls((1LL << (3 * d)) + 1);
  BBFMM_HIP_TRY(hipMemcpyAsync(ls.data(), t->leaf_start, ls.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  BBFMM_HIP_TRY(hipStreamSynchronize(s));
  std::vector<int> tgt;
  std::vector<long long> level_first(d + 2, 0);
  for (int l = 2; l <= d; ++l) {
    level_first[l] = (long long)tgt.size();
    const int sh = 3 * (d - l);
    const unsigned ncell = 1u << (3 * l);
    const int node_base = (int)(p->level_off[l] / nn);
    for (int o = 0; o < 8; ++o) {
      const int b = (int)tgt.size();
      for (unsigned c = (unsigned)o; c < ncell; c += 8)
        if (ls[(size_t)(c + 1) << sh] > ls[(size_t)c << sh]) tgt.push_back(node_base + (int)c);
      const int cnt = (int)tgt.size() - b;
      if (cnt == 0) continue;
      M2LLevel sg;
      std::memset(&sg, 0, sizeof(sg));
      sg.level = l;
      sg.side = 1 << l;
      sg.npar = cnt;
      sg.set = p->set_of_level[l];
      sg.scale = p->scale_of_level[l];
      sg.oct = o;
      sg.tgt_off = b;
      p->h_segs.push_back(sg);
    }
  }
  level_first[d + 1] = (long long)tgt.size();
  if (tgt.empty() || (long long)tgt.size() * kFarPerOctant > 0x7fffffffLL) {   // keep the dense path
    p->h_segs.clear();
    return BBFMM_OK;
  }
  hipError_t e = dmalloc(&p->d_utgt, tgt.size(), bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d_utgt, tgt.data(), tgt.size() * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = dmalloc(&p->d_uvsrc, tgt.size() * kFarPerOctant, bytes);
  for (int l = 2; l <= d && e == hipSuccess; ++l) {
    const int ntgt = (int)(level_first[l + 1] - level_first[l]);
    e = launch_uniform_vsrc(t->leaf_start, d, l, p->d_utgt + level_first[l], ntgt, (int)(p->level_off[l] / nn),
                            p->d_tab, p->d_uvsrc + level_first[l] * kFarPerOctant, s);
  }
  if (e == hipSuccess) e = hipMalloc((void**)&p->d_segs, p->h_segs.size() * sizeof(M2LLevel));
  if (e == hipSuccess) *bytes += (long long)(p->h_segs.size() * sizeof(M2LLevel));
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dfree(p->d_utgt); dfree(p->d_uvsrc); dfree(p->d_segs);
    p->d_utgt = nullptr; p->d_uvsrc = nullptr; p->d_segs = nullptr;
    p->h_segs.clear();
    return fail(e == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,
                std::string("M2L lists: ") + hipGetErrorString(e));
  }
  p->sparse_m2l = true;
  p->m2l_tgt = p->d_utgt;
  p->m2l_vsrc = p->d_uvsrc;
  return BBFMM_OK;
}

// Device build of an adaptive tree: keys, stable radix sort, sorted coordinates, then one
// segmentation step per level (cells of the level among the points still to be split), whose
// cells are copied to the host for the topology and lists.
bbfmm_status build_adaptive(std::unique_ptr<bbfmm_tree>& t, const double* d_points, long long n, int max_pts,
                            hipStream_t s, bbfmm_tree** out) {
  t->adaptive = true;
  t->max_leaf_points = max_pts;
  long long bytes = 0;
  unsigned long long *keys = nullptr, *ktmp = nullptr, *nkey = nullptr;
  int *vtmp = nullptr, *sflag = nullptr, *eflag = nullptr, *sidx = nullptr, *eidx = nullptr;
  int *nstart = nullptr, *nend = nullptr;
  unsigned char* active = nullptr;
  auto cleanup = [&]() {
    dfree(keys); dfree(ktmp); dfree(nkey); dfree(vtmp); dfree(sflag); dfree(eflag); dfree(sidx);
    dfree(eidx); dfree(nstart); dfree(nend); dfree(active);
  };
  auto bad = [&](hipError_t err, const char* what) {
    cleanup();
    free_tree_arrays(t.get());
    return fail(err == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,
                std::string(what) + ": " + hipGetErrorString(err));
  };
  hipError_t e = hipSuccess;
  if ((e = dmalloc(&t->xs, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->ys, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->zs, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->perm, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->leaf_of, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&keys, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&ktmp, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&nkey, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&vtmp, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&sflag, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&eflag, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&sidx, n + 1, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&eidx, n + 1, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&nstart, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&nend, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&active, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = launch_keys64(d_points, n, t->lo, t->width, keys, t->perm, s)) != hipSuccess) return bad(e, "keys");
  if ((e = radix_sort64(keys, t->perm, ktmp, vtmp, n, 3 * kAdaptiveDepth, s)) != hipSuccess)
    return bad(e, "sort");
  if ((e = launch_sorted_soa(d_points, t->perm, n, t->xs, t->ys, t->zs, s)) != hipSuccess)
    return bad(e, "sorted coordinates");
  if ((e = hipMemsetAsync(active, 1, n, s)) != hipSuccess) return bad(e, "memset");
  std::vector<std::vector<unsigned long long>> hkeys;
  std::vector<std::vector<int>> hstart, hend;
  int node_base = 0;
  for (int l = 0; l <= kAdaptiveDepth; ++l) {
    if ((e = launch_seg_flags(keys, n, l, active, sflag, eflag, s)) != hipSuccess) return bad(e, "segment");
    if ((e = exclusive_scan(sflag, sidx, n, s)) != hipSuccess) return bad(e, "scan");
    if ((e = exclusive_scan(eflag, eidx, n, s)) != hipSuccess) return bad(e, "scan");
    int cnt = 0;
    if ((e = hipMemcpyAsync(&cnt, sidx + n, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return bad(e, "count");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "count");
    if (cnt == 0) break;
    if ((long long)node_base + cnt > 0x7fffffffLL) {
      cleanup();
      free_tree_arrays(t.get());
      return fail(BBFMM_EUNSUPPORTED, "too many tree cells");
    }
    if ((e = launch_seg_compact(keys, n, l, sflag, sidx, eflag, eidx, nkey, nstart, nend, s)) != hipSuccess)
      return bad(e, "segment");
    hkeys.emplace_back(cnt);
    hstart.emplace_back(cnt);
    hend.emplace_back(cnt);
    if ((e = hipMemcpyAsync(hkeys.back().data(), nkey, cnt * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            s)) != hipSuccess)
      return bad(e, "copy");
    if ((e = hipMemcpyAsync(hstart.back().data(), nstart, cnt * sizeof(int), hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
      return bad(e, "copy");
    if ((e = hipMemcpyAsync(hend.back().data(), nend, cnt * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
      return bad(e, "copy");
    if ((e = launch_seg_next(n, l, max_pts, node_base, sidx, sflag, nstart, nend, active, t->leaf_of, s)) !=
        hipSuccess)
      return bad(e, "segment");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "segment");
    node_base += cnt;
  }
  cleanup();
  std::vector<int> grp;
  const std::vector<int> tab = octant_tables(&grp);
  try {
    build_adaptive_topology(t->topo, hkeys, hstart, hend, max_pts, t->lo, t->width, tab.data());
  } catch (const std::bad_alloc&) {
    free_tree_arrays(t.get());
    return fail(BBFMM_ENOMEM, "adaptive tree lists: host memory exhausted");
  }
  t->depth = t->topo.nlevels - 1;
  if ((e = upload_topology(t.get(), &bytes)) != hipSuccess) {
    free_tree_arrays(t.get());
    return fail(e == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,
                std::string("topology upload: ") + hipGetErrorString(e));
  }
  t->bytes = bytes;
  *out = t.release();
  return BBFMM_OK;
}

}  // namespace

bbfmm_status run_chain_work(bbfmm_plan* p, const double* in, int nrhs, double* out, const Work& wk,
                            hipStream_t s) {
  return run_chain_in(p, in, nrhs, out, wk, s);
}

// A plan holds one set of work buffers. A call on another stream than the plan's last call may
// start only once that call has completed; calls on the same stream are ordered by the stream.
bbfmm_status begin_call(bbfmm_plan* p, hipStream_t s) {
  if (!p->busy_set || p->busy_stream == s) return BBFMM_OK;
  const hipError_t q = hipEventQuery(p->busy);
  if (q == hipErrorNotReady)
    return fail(BBFMM_ESTATE, "the plan's previous call on another stream has not completed (one call at a time "
                              "per plan; synchronise that stream first)");
  if (q != hipSuccess) return fail(BBFMM_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(q));
  return BBFMM_OK;
}

bbfmm_status end_call(bbfmm_plan* p, hipStream_t s, bbfmm_status st) {
  if (st != BBFMM_OK) return st;
  if (!p->busy) BBFMM_HIP_TRY(hipEventCreateWithFlags(&p->busy, hipEventDisableTiming));
  BBFMM_HIP_TRY(hipEventRecord(p->busy, s));
  p->busy_stream = s;
  p->busy_set = true;
  return BBFMM_OK;
}

bbfmm_status check_apply_args(const bbfmm_plan* p, const double* in, int32_t nrhs,
                                     const double* out) {
  if (!p) return fail(BBFMM_EINVAL, "plan is null");
  if (!in || !out) return fail(BBFMM_EINVAL, "null input or output");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(BBFMM_EINVAL, "nrhs must be in [1, 64]");
  if (in == out) return fail(BBFMM_EINVAL, "input and output must not alias");
  return BBFMM_OK;
}

}  // namespace bbfmm

using namespace bbfmm;

extern "C" {

const char* bbfmm_last_error(void) { return g_last_error.c_str(); }
const char* bbfmm_version(void) { return "bbfmm-gfx950 0.1"; }

bbfmm_status bbfmm_build_octree(const double* d_points, int64_t n, const bbfmm_tree_opts* opts,
                                void* stream, bbfmm_tree** out) {
  if (!out) return fail(BBFMM_EINVAL, "out is null");
  *out = nullptr;
  if (!d_points || !opts) return fail(BBFMM_EINVAL, "null points or options");
  if (n < 1 || n > 0x7fffffffLL) return fail(BBFMM_EINVAL, "n must be in [1, 2^31 - 1]");
  const bool adaptive = opts->depth == -1;
  if (opts->depth < -1 || opts->depth > kMaxDepth)
    return fail(BBFMM_EINVAL, "depth must be in [0, 8], or -1 for an adaptive tree");
  if (adaptive && opts->max_leaf_points < 1)
    return fail(BBFMM_EINVAL, "max_leaf_points must be >= 1 for an adaptive tree");
  if (!adaptive && opts->max_leaf_points != 0)
    return fail(BBFMM_EINVAL, "max_leaf_points must be 0 for a uniform tree");
  if (opts->root_width > 0) {
    for (int r = 0; r < 3; ++r)
      if (!std::isfinite(opts->root_lo[r])) return fail(BBFMM_EINVAL, "root_lo is not finite");
    if (!std::isfinite(opts->root_width)) return fail(BBFMM_EINVAL, "root_width is not finite");
  }
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<bbfmm_tree> t(new (std::nothrow) bbfmm_tree());
  if (!t) return fail(BBFMM_ENOMEM, "host allocation");
  BBFMM_HIP_TRY(hipGetDevice(&t->device));
  t->n = n;
  t->depth = opts->depth;
  // Bounding box and validation (one synchronisation).
  const int nparts = bbox_parts(n);
  BBox* d_bb = nullptr;
  BBFMM_HIP_TRY(hipMalloc((void**)&d_bb, (nparts + 1) * sizeof(BBox)));
  BBox bb;
  hipError_t e = launch_bbox(d_points, n, d_bb + 1, nparts, d_bb, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&bb, d_bb, sizeof(BBox), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_bb);
  if (e != hipSuccess) return fail(BBFMM_EHIP, std::string("bounding box: ") + hipGetErrorString(e));
  if (bb.nonfinite > 0) return fail(BBFMM_EINVAL, "points contain non-finite coordinates");
  {
    const bbfmm_status st = root_of(bb.lo, bb.hi, opts->root_lo, opts->root_width, t.get());
    if (st != BBFMM_OK) return st;
  }
  if (adaptive) return build_adaptive(t, d_points, n, opts->max_leaf_points, s, out);
  const long long nleaf = 1LL << (3 * t->depth);
  long long bytes = 0;
  unsigned* keys = nullptr;
  int *counts = nullptr, *cursor = nullptr, *tmp = nullptr;
  auto cleanup = [&]() {
    dfree(keys); dfree(counts); dfree(cursor); dfree(tmp);
  };
  auto bad = [&](hipError_t err, const char* what) {
    cleanup();
    dfree(t->xs); dfree(t->ys); dfree(t->zs); dfree(t->perm); dfree(t->leaf_of); dfree(t->leaf_start);
    return fail(err == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,
                std::string(what) + ": " + hipGetErrorString(err));
  };
  if ((e = dmalloc(&t->xs, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->ys, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->zs, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->perm, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->leaf_of, n, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&t->leaf_start, nleaf + 1, &bytes)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&keys, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&counts, nleaf, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&cursor, nleaf, nullptr)) != hipSuccess) return bad(e, "alloc");
  if ((e = dmalloc(&tmp, n, nullptr)) != hipSuccess) return bad(e, "alloc");
  const double wleaf = t->width / (double)(1 << t->depth);
  if ((e = hipMemsetAsync(counts, 0, nleaf * sizeof(int), s)) != hipSuccess) return bad(e, "memset");
  if ((e = hipMemsetAsync(cursor, 0, nleaf * sizeof(int), s)) != hipSuccess) return bad(e, "memset");
  if ((e = launch_leaf_keys(d_points, n, t->lo, wleaf, t->depth, keys, counts, s)) != hipSuccess)
    return bad(e, "leaf keys");
  if ((e = exclusive_scan(counts, t->leaf_start, nleaf, s)) != hipSuccess) return bad(e, "scan");
  if ((e = launch_scatter(keys, n, t->leaf_start, cursor, tmp, s)) != hipSuccess) return bad(e, "scatter");
  if ((e = launch_order(d_points, keys, n, t->leaf_start, tmp, t->perm, t->leaf_of, t->xs, t->ys,
                        t->zs, s)) != hipSuccess)
    return bad(e, "order");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "build");
  cleanup();
  t->bytes = bytes;
  *out = t.release();
  return BBFMM_OK;
}

bbfmm_status bbfmm_tree_update_points(bbfmm_tree* t, const double* d_points, void* stream) {
  if (!t || !d_points) return fail(BBFMM_EINVAL, "null tree or points");
  if (t->adaptive) return fail(BBFMM_EUNSUPPORTED, "moving the points of an adaptive tree");
  if (!t->xs) return fail(BBFMM_ESTATE, "host-only tree");
  hipStream_t s = (hipStream_t)stream;
  if (!t->d_move_flag) BBFMM_HIP_TRY(dmalloc(&t->d_move_flag, 1, &t->bytes));
  unsigned bad = 0;
  const double wleaf = t->width / (double)(1 << t->depth);
  BBFMM_HIP_TRY(hipMemsetAsync(t->d_move_flag, 0, sizeof(unsigned), s));
  BBFMM_HIP_TRY(launch_move_check(d_points, t->n, t->perm, t->leaf_of, t->lo, wleaf, t->depth, t->d_move_flag, s));
  BBFMM_HIP_TRY(hipMemcpyAsync(&bad, t->d_move_flag, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  BBFMM_HIP_TRY(hipStreamSynchronize(s));
  if (bad != 0)
    return fail(BBFMM_EINVAL, std::to_string(bad) + " points left their leaf or the root cube (or are not finite)");
  BBFMM_HIP_TRY(launch_move_write(d_points, t->n, t->perm, t->xs, t->ys, t->zs, s));
  return BBFMM_OK;
}

void bbfmm_tree_destroy(bbfmm_tree* t) {
  if (!t) return;
  free_tree_arrays(t);
  delete t;
}

static bbfmm_status bbfmm_precompute_m2l_body(const bbfmm_tree* tree, const bbfmm_plan_opts* opts, void* stream, bbfmm_plan** out) {
  if (!out) return fail(BBFMM_EINVAL, "out is null");
  *out = nullptr;
  if (!tree || !opts) return fail(BBFMM_EINVAL, "null tree or options");
  if (!valid_kernel(opts->kernel)) return fail(BBFMM_EINVAL, "unknown kernel");
  if (opts->kernel == kInvSqrtR2C2 && !(opts->c > 0.0 && std::isfinite(opts->c)))
    return fail(BBFMM_EINVAL, "c must be finite and > 0 for 1/sqrt(r^2 + c^2)");
  if ((opts->kernel == kHelmCos || opts->kernel == kHelmSin) && !(opts->c >= 0.0 && std::isfinite(opts->c)))
    return fail(BBFMM_EINVAL, "the wavenumber c must be finite and >= 0");
  if (opts->m2l_prec < 0 || opts->m2l_prec > 2) return fail(BBFMM_EINVAL, "unknown M2L precision");
  if (!std::isfinite(opts->svd_eps)) return fail(BBFMM_EINVAL, "svd_eps is not finite");
  if (opts->compressor != BBFMM_COMPRESS_SVD && opts->compressor != BBFMM_COMPRESS_ACA)
    return fail(BBFMM_EINVAL, "unknown compressor");
  if (opts->variant != BBFMM_VARIANT_BLOCKED && opts->variant != BBFMM_VARIANT_SA &&
      opts->variant != BBFMM_VARIANT_SARCMP)
    return fail(BBFMM_EINVAL, "unknown M2L variant");
  if (opts->order < 2 || opts->order > kMaxOrder)
    return fail(BBFMM_EUNSUPPORTED, "order must be in [2, 9]");
  if (opts->order == 9 && opts->m2l_prec != BBFMM_M2L_FP64)
    return fail(BBFMM_EUNSUPPORTED, "order 9 runs the M2L in FP64 only");
  if (opts->order == 9 && opts->variant != BBFMM_VARIANT_BLOCKED)
    return fail(BBFMM_EUNSUPPORTED, "the SA variants run at orders up to 8");
  if (opts->variant != BBFMM_VARIANT_BLOCKED) {
    if (!(opts->svd_eps > 0)) return fail(BBFMM_EINVAL, "the SA variants need svd_eps > 0");
    if (tree->adaptive) return fail(BBFMM_EUNSUPPORTED, "the SA variants run on uniform trees");
    if (opts->m2l_prec != BBFMM_M2L_FP64) return fail(BBFMM_EUNSUPPORTED, "the SA variants run in FP64");
  }
  if (tree->adaptive && tree->xs == nullptr)
    return fail(BBFMM_ESTATE, "a host-only tree cannot be used for a plan");
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)stream;
  std::unique_ptr<bbfmm_plan> p(new (std::nothrow) bbfmm_plan());
  if (!p) return fail(BBFMM_ENOMEM, "host allocation");
  p->tree = tree;
  p->kernel = opts->kernel; p->c = opts->c; p->order = opts->order; p->eps = opts->svd_eps;
  p->prec = opts->m2l_prec;
  p->variant = opts->variant;
  const int L = p->order, nn = L * L * L, np = (nn + 15) / 16 * 16;
  p->nn = nn; p->np = np;
  const int depth = tree->depth;
  double degree = 0.0;
  const bool homog = kernel_is_homogeneous(p->kernel, &degree);
  p->nsets = depth >= 2 ? (homog ? 1 : depth - 1) : 0;
  for (int l = 2; l <= depth; ++l) {
    const double wl = tree->width / (double)(1 << l);
    p->set_of_level[l] = homog ? 0 : l - 2;
    p->scale_of_level[l] = homog ? std::pow(wl, degree) : 1.0;
  }
  // ---- operators (FP64 on the host) ----
  const int nsets = p->nsets;
  std::vector<std::vector<double>> kfull(nsets * kNumSym), ufac(nsets * kNumSym), vfac(nsets * kNumSym);
  p->ranks.assign(std::max(1, nsets) * kNumSym, nn);
  int max_rank = 0;
  for (int set = 0; set < nsets; ++set) {
    const double wset = homog ? 1.0 : tree->width / (double)(1 << (set + 2));
    for (int q = 0; q < kNumSym; ++q) {
      std::vector<double>& K = kfull[set * kNumSym + q];
      K.resize((size_t)nn * nn);
      m2l_operator(p->kernel, p->c, L, wset, q, K.data());
      if (p->eps > 0 && p->variant == BBFMM_VARIANT_BLOCKED) {
        std::vector<double>& Uf = ufac[set * kNumSym + q];
        std::vector<double>& Vf = vfac[set * kNumSym + q];
        const int r = compress_operator(K.data(), L, q, p->eps, opts->compressor, Uf, Vf);
        p->ranks[set * kNumSym + q] = r;
        max_rank = std::max(max_rank, r);
        // truncated operator for the full-rank fallback
        for (int i = 0; i < nn; ++i)
          for (int jj = 0; jj < nn; ++jj) {
            double acc = 0.0;
            for (int k = 0; k < r; ++k) acc += Uf[(size_t)i * r + k] * Vf[(size_t)jj * r + k];
            K[(size_t)i * nn + jj] = acc;
          }
      }
    }
  }
  p->lowrank = p->eps > 0 && p->variant == BBFMM_VARIANT_BLOCKED && nsets > 0 && L >= 3 &&
               max_rank <= m2l_ia_rank_limit(L);
  // SA / SArcmp: basis and cores of every operator set ([n][rp] basis, [r][n] transposed,
  // then the cores by offset code)
  std::vector<double> sblob;
  std::vector<long long> sa_off;
  if (p->variant != BBFMM_VARIANT_BLOCKED) {
    sa_off.assign((size_t)nsets * 512, 0);
    p->sa_rank_h.assign((size_t)nsets * 512, 0);
    for (int set = 0; set < nsets; ++set) {
      const double wset = homog ? 1.0 : tree->width / (double)(1 << (set + 2));
      SAOperators op;
      sa_operators(p->kernel, p->c, L, wset, p->eps, p->variant == BBFMM_VARIANT_SARCMP, op);
      const int r = op.r, rp = 16 * ((r + 15) / 16);
      if (r < 1 || r > kSAMaxRank) return fail(BBFMM_EUNSUPPORTED, "SA basis rank outside [1, 192]");
      p->sa_r.push_back(r);
      p->sa_rp.push_back(rp);
      p->sa_u_off.push_back((long long)sblob.size());
      for (int i = 0; i < nn; ++i)
        for (int k = 0; k < rp; ++k) sblob.push_back(k < r ? op.u[(size_t)i * r + k] : 0.0);
      p->sa_ut_off.push_back((long long)sblob.size());
      for (int k = 0; k < r; ++k)
        for (int i = 0; i < nn; ++i) sblob.push_back(op.u[(size_t)i * r + k]);
      int max_op = 0;
      for (int code = 0; code < 512; ++code) {
        const int rt = op.rank[code];
        p->sa_rank_h[(size_t)set * 512 + code] = rt;
        if (op.core[code].empty() && op.ubar[code].empty()) continue;
        max_op = std::max(max_op, rt == r ? rp * rp : 2 * rp * (16 * ((rt + 15) / 16)));
        sa_off[(size_t)set * 512 + code] = (long long)sblob.size();
        if (rt == r) {
          const std::vector<double>& C = op.core[code];     // C_t^T, [rp][rp]
          for (int k = 0; k < rp; ++k)
            for (int i = 0; i < rp; ++i) sblob.push_back(k < r && i < r ? C[(size_t)i * r + k] : 0.0);
        } else {
          const int rt16 = 16 * ((rt + 15) / 16);
          const std::vector<double>& ub = op.ubar[code];
          const std::vector<double>& vb = op.vbar[code];
          for (int k = 0; k < rp; ++k)                       // Vbar, [rp][rt16]
            for (int q = 0; q < rt16; ++q) sblob.push_back(k < r && q < rt ? vb[(size_t)k * rt + q] : 0.0);
          for (int q = 0; q < rt16; ++q)                     // Ubar^T, [rt16][rp]
            for (int i = 0; i < rp; ++i) sblob.push_back(i < r && q < rt ? ub[(size_t)i * rt + q] : 0.0);
        }
      }
      p->sa_max_op.push_back(max_op);
    }
  }
  p->h_k = kfull;
  p->h_u = ufac;
  p->h_v = vfac;
  // ---- device layout ----
  std::vector<double> blob;
  p->op_off.assign(std::max(1, nsets) * kNumSym * 2, 0);
  for (int set = 0; set < nsets; ++set)
    for (int q = 0; q < kNumSym; ++q) {
      const int idx = set * kNumSym + q;
      if (!p->lowrank) {
        p->op_off[idx * 2] = (long long)blob.size();
        blob.insert(blob.end(), kfull[idx].begin(), kfull[idx].end());
      } else {
        const int r = p->ranks[idx], ru = (r + 3) / 4 * 4, rv = (r + 15) / 16 * 16;
        p->op_off[idx * 2] = (long long)blob.size();
        for (int i = 0; i < nn; ++i)
          for (int k = 0; k < ru; ++k) blob.push_back(k < r ? ufac[idx][(size_t)i * r + k] : 0.0);
        p->op_off[idx * 2 + 1] = (long long)blob.size();
        for (int i = 0; i < nn; ++i)
          for (int k = 0; k < rv; ++k) blob.push_back(k < r ? vfac[idx][(size_t)i * r + k] : 0.0);
      }
    }
  std::vector<int> grp;
  std::vector<int> tab = octant_tables(&grp);
  p->h_tab = tab;
  p->h_grp = grp;
  std::vector<short> sig((size_t)kNumPerms * np), siginv((size_t)kNumPerms * np);
  {
    std::vector<int32_t> tmpv(nn);
    for (int pid = 0; pid < kNumPerms; ++pid) {
      sigma_table(L, pid, tmpv.data());
      for (int i = 0; i < np; ++i) {
        sig[(size_t)pid * np + i] = (short)(i < nn ? tmpv[i] : nn);
        siginv[(size_t)pid * np + i] = (short)nn;
      }
      for (int i = 0; i < nn; ++i) siginv[(size_t)pid * np + tmpv[i]] = (short)i;
    }
  }
  const std::vector<double> x = cheb_nodes(L);
  std::vector<double> tk((size_t)L * L), m2m((size_t)2 * L * L);
  for (int k = 0; k < L; ++k)
    for (int m = 0; m < L; ++m) tk[(size_t)k * L + m] = std::cos(k * std::acos(x[m]));
  for (int sbit = 0; sbit < 2; ++sbit)
    for (int bc = 0; bc < L; ++bc)
      for (int bp = 0; bp < L; ++bp)
        m2m[((size_t)sbit * L + bc) * L + bp] = cheb_basis(L, 0.5 * (2 * sbit - 1) + 0.5 * x[bc], bp);
  // ---- upload ----
  long long bytes = 0;
  auto up = [&](void** dst, const void* src, size_t nbytes) -> hipError_t {
    *dst = nullptr;
    if (nbytes == 0) return hipSuccess;
    hipError_t er = hipMalloc(dst, nbytes);
    if (er != hipSuccess) return er;
    bytes += (long long)nbytes;
    return hipMemcpyAsync(*dst, src, nbytes, hipMemcpyHostToDevice, s);
  };
  auto destroy_partial = [&]() {
    dfree(p->ops_hi); dfree(p->ops_lo); dfree(p->d_op_off); dfree(p->d_op_rank); dfree(p->d_tab);
    dfree(p->d_grp); dfree(p->d_sig); dfree(p->d_siginv); dfree(p->d_tk); dfree(p->d_m2m);
    dfree(p->d_zeros); dfree(p->d_sa); dfree(p->d_sa_off); dfree(p->d_sa_rank);
  };
  hipError_t e = hipSuccess;
  std::vector<float> hi, lo;
  if (p->prec == 0) {
    e = up(&p->ops_hi, blob.data(), blob.size() * sizeof(double));
  } else {
    hi.resize(blob.size());
    lo.resize(blob.size());
    for (size_t i = 0; i < blob.size(); ++i) {
      hi[i] = (float)blob[i];
      lo[i] = (float)(blob[i] - (double)hi[i]);
    }
    e = up(&p->ops_hi, hi.data(), hi.size() * sizeof(float));
    if (e == hipSuccess && p->prec == 2) e = up(&p->ops_lo, lo.data(), lo.size() * sizeof(float));
  }
  if (e == hipSuccess) e = up((void**)&p->d_op_off, p->op_off.data(), p->op_off.size() * sizeof(long long));
  if (e == hipSuccess) e = up((void**)&p->d_op_rank, p->ranks.data(), p->ranks.size() * sizeof(int));
  if (e == hipSuccess) e = up((void**)&p->d_tab, tab.data(), tab.size() * sizeof(int));
  if (e == hipSuccess) e = up((void**)&p->d_grp, grp.data(), grp.size() * sizeof(int));
  if (e == hipSuccess) e = up((void**)&p->d_sig, sig.data(), sig.size() * sizeof(short));
  if (e == hipSuccess) e = up((void**)&p->d_siginv, siginv.data(), siginv.size() * sizeof(short));
  if (e == hipSuccess) e = up((void**)&p->d_tk, tk.data(), tk.size() * sizeof(double));
  if (e == hipSuccess) e = up((void**)&p->d_m2m, m2m.data(), m2m.size() * sizeof(double));
  p->h_m2m = m2m;
  const std::vector<double> zeros((size_t)nn * kMaxRhs, 0.0);
  if (e == hipSuccess) e = up((void**)&p->d_zeros, zeros.data(), zeros.size() * sizeof(double));
  if (e == hipSuccess && p->variant != BBFMM_VARIANT_BLOCKED) {
    e = up((void**)&p->d_sa, sblob.data(), sblob.size() * sizeof(double));
    if (e == hipSuccess) e = up((void**)&p->d_sa_off, sa_off.data(), sa_off.size() * sizeof(long long));
    if (e == hipSuccess) e = up((void**)&p->d_sa_rank, p->sa_rank_h.data(), p->sa_rank_h.size() * sizeof(int));
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    destroy_partial();
    return fail(e == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,
                std::string("precompute upload: ") + hipGetErrorString(e));
  }
  if (tree->adaptive) {
    // M2L segments: the targets of one (level, octant); tiles are set per nrhs at apply time
    const AdaptiveTopology& T = tree->topo;
    for (int l = 2; l < T.nlevels; ++l)
      for (int o = 0; o < 8; ++o) {
        const int b = T.m2l_off[l * 8 + o], e2 = T.m2l_off[l * 8 + o + 1];
        if (e2 == b) continue;
        M2LLevel sg;
        std::memset(&sg, 0, sizeof(sg));
        sg.level = l;
        sg.side = 1 << std::min(l, 30);
        sg.npar = e2 - b;
        sg.set = p->set_of_level[l];
        sg.scale = p->scale_of_level[l];
        sg.oct = o;
        sg.tgt_off = b;
        p->h_segs.push_back(sg);
      }
    if (!p->h_segs.empty() && e == hipSuccess) {
      e = hipMalloc((void**)&p->d_segs, p->h_segs.size() * sizeof(M2LLevel));
      if (e == hipSuccess) bytes += (long long)(p->h_segs.size() * sizeof(M2LLevel));
    }
    if (e != hipSuccess) {
      destroy_partial();
      return fail(e == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,
                  std::string("precompute upload: ") + hipGetErrorString(e));
    }
    p->exp_elems = (long long)T.key.size() * nn;
    p->m2l_tgt = tree->d_m2l_tgt;
    p->m2l_vsrc = tree->d_vsrc;
  } else {
    long long off = 0;
    for (int l = 2; l <= depth; ++l) {
      p->level_off[l] = off;
      off += (1LL << (3 * l)) * nn;
    }
    p->exp_elems = off;
    // compressed operators: scratch for splitting the M2L's last round of workgroups
    if (p->lowrank && depth >= 2) {
      int dev = 0, cus = 0;
      hipError_t e2 = hipGetDevice(&dev);
      if (e2 == hipSuccess) e2 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      const int slots = 2 * cus;       // resident compressed-kernel workgroups at most
      if (e2 == hipSuccess && slots > 0) {
        p->split_cap = m2l_split_scratch_doubles(L, slots);
        p->tcount_len = slots / 2;
        e2 = dmalloc(&p->d_split, (size_t)p->split_cap, &bytes);
        if (e2 == hipSuccess) e2 = dmalloc(&p->d_tcount, (size_t)p->tcount_len, &bytes);
        if (e2 == hipSuccess) e2 = hipMemset(p->d_tcount, 0, sizeof(unsigned) * p->tcount_len);
      }
      if (e2 != hipSuccess) {
        destroy_partial();
        dfree(p->d_split); dfree(p->d_tcount);
        return fail(e2 == hipErrorOutOfMemory ? BBFMM_ENOMEM : BBFMM_EHIP,
                    std::string("M2L scratch: ") + hipGetErrorString(e2));
      }
    }
    // full-rank operators: M2L over the targets that hold points only
    if (!p->lowrank && p->variant == BBFMM_VARIANT_BLOCKED && depth >= 2) {
      const bbfmm_status st = build_sparse_uniform(p.get(), s, &bytes);
      if (st != BBFMM_OK) {
        destroy_partial();
        return st;
      }
    }
  }
  p->op_bytes = bytes;
  p->precompute_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = p.release();
  return BBFMM_OK;
}

// Host allocations of the precompute that fail (std::bad_alloc) return BBFMM_ENOMEM rather than
// crossing the C ABI; device allocations report their own errors.
bbfmm_status bbfmm_precompute_m2l(const bbfmm_tree* tree, const bbfmm_plan_opts* opts,
                                  void* stream, bbfmm_plan** out) {
  try {
    return bbfmm_precompute_m2l_body(tree, opts, stream, out);
  } catch (const std::bad_alloc&) {
    if (out) *out = nullptr;
    return fail(BBFMM_ENOMEM, "operator precompute: host memory exhausted");
  }
}

void bbfmm_plan_destroy(bbfmm_plan* p) {
  if (!p) return;
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->busy) (void)hipEventDestroy(p->busy);
  free_buffers(p);
  dfree(p->cplx_q); dfree(p->cplx_a); dfree(p->cplx_b);
  dfree(p->ops_hi); dfree(p->ops_lo); dfree(p->d_op_off); dfree(p->d_op_rank); dfree(p->d_tab);
  dfree(p->d_grp); dfree(p->d_sig); dfree(p->d_siginv); dfree(p->d_tk); dfree(p->d_m2m);
  dfree(p->d_zeros); dfree(p->d_segs); dfree(p->d_utgt); dfree(p->d_uvsrc);
  dfree(p->d_split); dfree(p->d_tcount);
  dfree(p->d_abl_ops); dfree(p->d_abl_off); dfree(p->d_abl_rank);
  dfree(p->d_sa); dfree(p->d_sa_off); dfree(p->d_sa_rank);
  delete p;
}

bbfmm_status bbfmm_apply(bbfmm_plan* p, const double* d_q, int32_t nrhs, double* d_phi, void* stream) {
  bbfmm_status st = check_apply_args(p, d_q, nrhs, d_phi);
  if (st != BBFMM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = begin_call(p, s)) != BBFMM_OK) return st;
  return end_call(p, s, run_chain(p, d_q, nrhs, d_phi, 0, s));
}

bbfmm_status bbfmm_apply_adjoint(bbfmm_plan* p, const double* d_g, int32_t nrhs, double* d_grad_q,
                                 void* stream) {
  bbfmm_status st = check_apply_args(p, d_g, nrhs, d_grad_q);
  if (st != BBFMM_OK) return st;
  // The supported kernels are symmetric and sources = targets: L2P^T = P2M, L2L^T = M2M,
  // K_t^T = K_{-t} (so M2L^T is the M2L of the reversed pairs) and the near field is symmetric;
  // the transposed chain is therefore the forward pass sequence run on g.
  hipStream_t s = (hipStream_t)stream;
  if ((st = begin_call(p, s)) != BBFMM_OK) return st;
  return end_call(p, s, run_chain(p, d_g, nrhs, d_grad_q, 1, s));
}

bbfmm_status bbfmm_eval_grad(bbfmm_plan* p, const double* d_q, const double* d_g, int32_t nrhs,
                             int32_t roles, double* d_grad_x, void* stream) {
  if (!p) return fail(BBFMM_EINVAL, "plan is null");
  if (!d_q || !d_g || !d_grad_x) return fail(BBFMM_EINVAL, "null argument");
  if (roles < 1 || roles > 3) return fail(BBFMM_EINVAL, "roles must be 1, 2 or 3");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(BBFMM_EINVAL, "nrhs must be in [1, 64]");
  if (p->tree->adaptive) return fail(BBFMM_EUNSUPPORTED, "gradients are not supported on adaptive trees");
  if (p->slot_nrhs[0] != nrhs || p->slot_nrhs[1] != nrhs)
    return fail(BBFMM_ESTATE, "eval_grad needs bbfmm_apply(q) and bbfmm_apply_adjoint(g) with this nrhs first");
  hipStream_t s = (hipStream_t)stream;
  bbfmm_status st = begin_call(p, s);
  if (st != BBFMM_OK) return st;
  const bbfmm_tree* t = p->tree;
  const PassGeom g = geom_of(p);
  // densities in sorted order are already in qs[0] / qs[1] from the two chains; re-gather in case
  // the caller passes different arrays than were applied (they must be the same values).
  BBFMM_HIP_TRY(launch_gather_rows(d_q, t->perm, t->n, nrhs, p->qs[0], s));
  BBFMM_HIP_TRY(launch_gather_rows(d_g, t->perm, t->n, nrhs, p->qs[1], s));
  const double* Fq = t->depth >= 2 ? p->F[0] + p->level_off[t->depth] * nrhs : nullptr;
  const double* Fg = t->depth >= 2 ? p->F[1] + p->level_off[t->depth] * nrhs : nullptr;
  BBFMM_HIP_TRY(launch_grad(g, p->qs[0], p->qs[1], Fq, Fg, nrhs, roles, d_grad_x, s));
  return end_call(p, s, BBFMM_OK);
}

bbfmm_status bbfmm_helmholtz_apply(bbfmm_plan* re, bbfmm_plan* im, const double* d_q, int32_t nrhs,
                                   int32_t complex_q, double* d_phi, void* stream) {
  if (!re || !im) return fail(BBFMM_EINVAL, "plan is null");
  if (!d_q || !d_phi) return fail(BBFMM_EINVAL, "null input or output");
  if (d_q == d_phi) return fail(BBFMM_EINVAL, "input and output must not alias");
  if (complex_q != 0 && complex_q != 1) return fail(BBFMM_EINVAL, "complex_q must be 0 or 1");
  const int cols = complex_q ? 2 * nrhs : nrhs;
  if (nrhs < 1 || cols > kMaxRhs) return fail(BBFMM_EINVAL, "nrhs must be in [1, 64] (real q) or [1, 32] (complex q)");
  if (re == im) return fail(BBFMM_EINVAL, "the two plans must differ");
  if (re->kernel != BBFMM_K_HELM_COS || im->kernel != BBFMM_K_HELM_SIN)
    return fail(BBFMM_EINVAL, "re must be a cos(kr)/r plan and im a sin(kr)/r plan");
  if (re->tree != im->tree || re->c != im->c || re->order != im->order)
    return fail(BBFMM_EINVAL, "the two plans must share tree, order and wavenumber");
  hipStream_t s = (hipStream_t)stream;
  bbfmm_status st = begin_call(re, s);
  if (st == BBFMM_OK) st = begin_call(im, s);
  if (st != BBFMM_OK) return st;
  const long long n = re->tree->n;
  const long long need = n * cols;
  if (need > re->cplx_cap) {
    dfree(re->cplx_q); dfree(re->cplx_a); dfree(re->cplx_b);
    re->cplx_q = re->cplx_a = re->cplx_b = nullptr;
    re->cplx_cap = 0;
    BBFMM_HIP_TRY(dmalloc(&re->cplx_q, (size_t)need, nullptr));
    BBFMM_HIP_TRY(dmalloc(&re->cplx_a, (size_t)need, nullptr));
    BBFMM_HIP_TRY(dmalloc(&re->cplx_b, (size_t)need, nullptr));
    re->cplx_cap = need;
  }
  const double* in = d_q;
  if (complex_q) {
    BBFMM_HIP_TRY(launch_split_complex(d_q, n, nrhs, re->cplx_q, s));
    in = re->cplx_q;
  }
  st = run_chain(re, in, cols, re->cplx_a, 0, s);
  if (st == BBFMM_OK) st = run_chain(im, in, cols, re->cplx_b, 0, s);
  if (st != BBFMM_OK) return st;
  BBFMM_HIP_TRY(launch_combine_complex(re->cplx_a, re->cplx_b, n, nrhs, complex_q, d_phi, s));
  st = end_call(re, s, BBFMM_OK);
  return st != BBFMM_OK ? st : end_call(im, s, BBFMM_OK);
}

bbfmm_status bbfmm_plan_set_timing(bbfmm_plan* p, int32_t enable) {
  if (!p) return fail(BBFMM_EINVAL, "plan is null");
  p->timing = enable != 0;
  p->ev_used = 0;
  return BBFMM_OK;
}

bbfmm_status bbfmm_plan_pass_times(bbfmm_plan* p, double* out_ms, int32_t* out_calls) {
  if (!p || !out_ms) return fail(BBFMM_EINVAL, "null argument");
  for (int k = 0; k < kNumPasses; ++k) out_ms[k] = 0.0;
  int calls = 0;
  if (p->ev_used > 0) BBFMM_HIP_TRY(hipEventSynchronize(p->ev_pool[p->ev_used - 1]));
  for (size_t k = 0; k < p->ev_used; ++k) {
    if (p->ev_tag[k] == kPassStart) {
      ++calls;
      continue;
    }
    float ms = 0.0f;
    BBFMM_HIP_TRY(hipEventElapsedTime(&ms, p->ev_pool[k - 1], p->ev_pool[k]));
    out_ms[p->ev_tag[k]] += ms;
  }
  if (out_calls) *out_calls = calls;
  return BBFMM_OK;
}

bbfmm_status bbfmm_plan_stats(const bbfmm_plan* p, bbfmm_stats* out) {
  if (!p || !out) return fail(BBFMM_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  const bbfmm_tree* t = p->tree;
  out->n_points = t->n;
  out->depth = t->depth;
  out->order = p->order;
  out->n_levels_m2l = t->depth >= 2 ? t->depth - 1 : 0;
  out->n_operator_sets = p->nsets;
  for (int q = 0; q < kNumSym; ++q) out->rank[q] = p->eps > 0 ? p->ranks[q] : p->nn;
  out->m2l_kernel = p->variant != BBFMM_VARIANT_BLOCKED ? 2 : (p->lowrank ? 1 : 0);
  out->variant = p->variant;
  if (p->variant != BBFMM_VARIANT_BLOCKED && !p->sa_r.empty()) {
    out->sa_rank = p->sa_r[0];
    double sum = 0.0;
    int cnt = 0;
    for (int code = 0; code < 512; ++code)
      if (p->sa_rank_h[code] > 0) {
        sum += p->sa_rank_h[code];
        ++cnt;
      }
    out->sa_mean_core_rank = cnt ? sum / cnt : 0.0;
  }
  for (int r = 0; r < 3; ++r) out->root_lo[r] = t->lo[r];
  out->root_width = t->width;
  out->precompute_seconds = p->precompute_seconds;
  out->device_bytes = t->bytes + p->op_bytes + p->buffer_bytes;
  if (t->adaptive) {
    // V-list pairs by level and representative, from the host lists
    const AdaptiveTopology& T = t->topo;
    int nlev = 0;
    const double nn = p->nn;
    for (int l = 2; l < T.nlevels; ++l) {
      std::vector<long long> cnt(kNumSym, 0);
      bool any = false;
      for (int o = 0; o < 8; ++o)
        for (int slot = T.m2l_off[l * 8 + o]; slot < T.m2l_off[l * 8 + o + 1]; ++slot)
          for (int e = 0; e < kFarPerOctant; ++e)
            if (T.vsrc[(size_t)slot * kFarPerOctant + e] >= 0) {
              ++cnt[(p->h_tab[o * kFarPerOctant + e] >> 9) & 15];
              any = true;
            }
      nlev += any ? 1 : 0;
      const int set = p->set_of_level[l];
      for (int q = 0; q < kNumSym; ++q) {
        const double c = (double)cnt[q];
        out->pairs_total += cnt[q];
        out->pairs_nonempty += cnt[q];
        const double r = p->ranks[set * kNumSym + q];
        out->m2l_flops_algorithmic += c * (p->lowrank ? 4.0 * nn * r : 2.0 * nn * nn);
      }
      // issued: every tile of 64 columns runs every transfer vector of its octant
      for (int o = 0; o < 8; ++o) {
        const double targets = T.m2l_off[l * 8 + o + 1] - T.m2l_off[l * 8 + o];
        for (int q = 0; q < kNumSym; ++q) {
          const int np_q = p->h_grp[o * 17 + q + 1] - p->h_grp[o * 17 + q];
          const double per_t = m2l_issued_flops_per_t(p->order, p->lowrank, p->ranks[set * kNumSym + q]);
          out->m2l_flops_issued += targets / 64.0 * np_q * per_t;
        }
      }
    }
    out->n_levels_m2l = nlev;
    return BBFMM_OK;
  }
  if (t->depth < 2) return BBFMM_OK;
  unsigned long long* d_counts = nullptr;
  const int nlev = t->depth - 1;
  BBFMM_HIP_TRY(hipMalloc((void**)&d_counts, sizeof(unsigned long long) * 16 * nlev));
  hipError_t e = hipMemset(d_counts, 0, sizeof(unsigned long long) * 16 * nlev);
  for (int l = 2; l <= t->depth && e == hipSuccess; ++l)
    e = launch_count_pairs(t->leaf_start, t->depth, l, p->d_tab, d_counts + 16 * (l - 2), nullptr);
  std::vector<unsigned long long> counts(16 * nlev);
  if (e == hipSuccess)
    e = hipMemcpy(counts.data(), d_counts, counts.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
  (void)hipFree(d_counts);
  if (e != hipSuccess) return fail(BBFMM_EHIP, std::string("plan_stats: ") + hipGetErrorString(e));
  const double nn = p->nn;
  for (int l = 2; l <= t->depth; ++l) {
    const long long s = 1LL << l;
    out->pairs_total += (6 * s - 8) * (6 * s - 8) * (6 * s - 8) - (3 * s - 2) * (3 * s - 2) * (3 * s - 2);
    const int set = p->set_of_level[l];
    if (p->variant != BBFMM_VARIANT_BLOCKED) {
      // SA: every in-box pair at its core's cost, plus projection and expansion of every cell
      for (int q = 0; q < kNumSym; ++q) out->pairs_nonempty += (long long)counts[16 * (l - 2) + q];
      const int r = p->sa_r[set], rp = p->sa_rp[set];
      const double ncell = (double)(1LL << (3 * l));
      out->m2l_flops_algorithmic += ncell * 4.0 * nn * r;
      out->m2l_flops_issued += ncell * 2.0 * nn * (rp + r);
      for (int o = 0; o < 8; ++o) {
        const double tiles = (double)(1LL << (3 * (l - 1))) / 64.0;
        for (int e = 0; e < kFarPerOctant; ++e) {
          const int code = p->h_tab[o * kFarPerOctant + e] & 511;
          double cnt = 1.0;
          for (int ax = 0; ax < 3; ++ax) {
            const int d = ((code >> (3 * ax)) & 7) - 3, bit = (o >> ax) & 1;
            long long c = 0;
            for (long long x = bit; x < s; x += 2) c += (x + d >= 0 && x + d < s) ? 1 : 0;
            cnt *= (double)c;
          }
          const int rt = p->sa_rank_h[(size_t)set * 512 + code];
          out->m2l_flops_algorithmic += cnt * (rt == r ? 2.0 * r * r : 4.0 * r * rt);
          double mfma = 0.0;
          if (rt == r) {
            mfma = (rp / 4.0) * (rp / 16);
          } else {
            for (int b2 = 0; 16 * b2 < rt; ++b2) mfma += rp / 4.0 + std::min(4, (rt - 16 * b2 + 3) / 4) * (rp / 16);
          }
          out->m2l_flops_issued += tiles * 4.0 * mfma * 2048.0;
        }
      }
      continue;
    }
    for (int q = 0; q < kNumSym; ++q) {
      const double c = (double)counts[16 * (l - 2) + q];
      out->pairs_nonempty += (long long)c;
      const double r = p->ranks[set * kNumSym + q];
      out->m2l_flops_algorithmic += c * (p->lowrank ? 4.0 * nn * r : 2.0 * nn * nn);
    }
    // issued: every tile runs every transfer vector of its octant (upper bound for the segment
    // path, which skips transfer vectors without a source in the tile)
    for (int o = 0; o < 8; ++o) {
      double targets = (double)(1LL << (3 * (l - 1)));
      if (p->sparse_m2l) {
        targets = 0;
        for (const M2LLevel& sg : p->h_segs)
          if (sg.level == l && sg.oct == o) targets += sg.npar;
      }
      for (int q = 0; q < kNumSym; ++q) {
        const int np_q = p->h_grp[o * 17 + q + 1] - p->h_grp[o * 17 + q];
        const double per_t = m2l_issued_flops_per_t(p->order, p->lowrank, p->ranks[set * kNumSym + q]);
        out->m2l_flops_issued += targets / 64.0 * np_q * per_t;
      }
    }
  }
  return BBFMM_OK;
}

bbfmm_status bbfmm_debug_get_expansions(const bbfmm_plan* p, int32_t level, int32_t which, int32_t nrhs_out,
                                        double* d_out, void* stream) {
  if (!p || !d_out) return fail(BBFMM_EINVAL, "null argument");
  const bbfmm_tree* t = p->tree;
  if (t->adaptive) return fail(BBFMM_EUNSUPPORTED, "uniform trees only");
  if (level < 2 || level > t->depth) return fail(BBFMM_EINVAL, "level must be in [2, depth]");
  if (which < 0 || which > 2) return fail(BBFMM_EINVAL, "which must be 0, 1 or 2");
  const int nrhs = p->slot_nrhs[0];
  if (nrhs == 0 || !p->W) return fail(BBFMM_ESTATE, "no apply has run on this plan");
  if (nrhs_out != nrhs)
    return fail(BBFMM_EINVAL, "nrhs " + std::to_string(nrhs_out) + " differs from the last apply's " +
                                  std::to_string(nrhs));
  const size_t count = (size_t)(1LL << (3 * level)) * p->nn * nrhs;
  const double* src = nullptr;
  if (which == 0) src = p->W + p->level_off[level] * nrhs;
  else src = p->F[0] + p->level_off[level] * nrhs;
  if (which == 1) {
    // M2L output alone: rerun the M2L of this level into the output
    const M2LArgs a = m2l_args(p, nrhs, p->W + p->level_off[level] * nrhs, d_out, level);
    BBFMM_HIP_TRY(launch_m2l(p->order, p->lowrank, p->prec, a, (hipStream_t)stream));
    return BBFMM_OK;
  }
  BBFMM_HIP_TRY(hipMemcpyAsync(d_out, src, count * sizeof(double), hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
  return BBFMM_OK;
}

bbfmm_status bbfmm_debug_m2l_level(bbfmm_plan* p, int32_t level, const double* d_w, int32_t nrhs,
                                   double* d_f, void* stream) {
  if (!p || !d_w || !d_f) return fail(BBFMM_EINVAL, "null argument");
  if (p->tree->adaptive) return fail(BBFMM_EUNSUPPORTED, "uniform trees only");
  if (level < 2 || level > p->tree->depth) return fail(BBFMM_EINVAL, "level must be in [2, depth]");
  if (nrhs < 1 || nrhs > kMaxRhs) return fail(BBFMM_EINVAL, "nrhs must be in [1, 64]");
  hipStream_t s = (hipStream_t)stream;
  bbfmm_status st = begin_call(p, s);
  if (st != BBFMM_OK) return st;
  if (p->variant != BBFMM_VARIANT_BLOCKED) {
    st = ensure_buffers(p, nrhs, 0);
    if (st != BBFMM_OK) return st;
    return end_call(p, s, sa_levels(p, nrhs, d_w, d_f, level, s));
  }
  const M2LArgs a = m2l_args(p, nrhs, d_w, d_f, level);
  BBFMM_HIP_TRY(launch_m2l(p->order, p->lowrank, p->prec, a, s));
  return end_call(p, s, BBFMM_OK);
}

bbfmm_status bbfmm_m2l_unblocked(bbfmm_plan* p, int32_t level, int32_t variant, const double* d_w,
                                 int32_t nrhs, double* d_f, void* stream) {
  if (!p || !d_w || !d_f) return fail(BBFMM_EINVAL, "null argument");
  if (p->tree->adaptive) return fail(BBFMM_EUNSUPPORTED, "uniform trees only");
  if (level < 2 || level > p->tree->depth) return fail(BBFMM_EINVAL, "level must be in [2, depth]");
  if (variant < 0 || variant > 3) return fail(BBFMM_EINVAL, "variant must be 0 (NA), 1 (NAsym), 2 (IA) or 3 (IAsym)");
  if (nrhs != 1 && nrhs != 2 && nrhs != 4) return fail(BBFMM_EINVAL, "nrhs must be 1, 2 or 4");
  const bool lowrank_variant = variant >= 2;
  if (lowrank_variant && !(p->eps > 0)) return fail(BBFMM_EUNSUPPORTED, "IA variants need a compressed plan");
  const int L = p->order, nn = p->nn, np = p->np;
  const int set = p->set_of_level[level];
  if (lowrank_variant)
    for (int q = 0; q < kNumSym; ++q)
      if (p->ranks[set * kNumSym + q] > 64) return fail(BBFMM_EUNSUPPORTED, "ranks above 64");
  hipStream_t s = (hipStream_t)stream;
  const bbfmm_status st0 = begin_call(p, s);
  if (st0 != BBFMM_OK) return st0;
  if (p->abl_variant != variant || p->abl_set != set) {
    // operators of the variant on the host, transposed, then uploaded
    const bool sym = variant == 1 || variant == 3;
    const int nidx = sym ? kNumSym : 512;       // representatives, or offset codes of t
    std::vector<double> blob;
    std::vector<long long> off(2 * (size_t)nidx, 0);
    std::vector<int> rank(nidx, 0);
    std::vector<int32_t> sg(nn);
    for (int idx = 0; idx < nidx; ++idx) {
      int q = idx;
      if (!sym) {
        const int t[3] = {-((idx & 7) - 3), -(((idx >> 3) & 7) - 3), -(((idx >> 6) & 7) - 3)};
        const int linf = std::max(std::abs(t[0]), std::max(std::abs(t[1]), std::abs(t[2])));
        if ((idx & 7) > 6 || ((idx >> 3) & 7) > 6 || ((idx >> 6) & 7) > 6 || linf < 2) continue;
        const SymInfo si = symmetry_of(t);
        q = si.p;
        sigma_table(L, si.perm_id, sg.data());
      } else {
        for (int i = 0; i < nn; ++i) sg[i] = i;
      }
      const int opi = set * kNumSym + q;
      if (!lowrank_variant) {
        const std::vector<double>& K = p->h_k[opi];
        off[2 * idx] = (long long)blob.size();
        for (int j = 0; j < nn; ++j)
          for (int i = 0; i < nn; ++i) blob.push_back(K[(size_t)sg[i] * nn + sg[j]]);   // K_t^T
      } else {
        const int r = p->ranks[opi];
        rank[idx] = r;
        const std::vector<double>& U = p->h_u[opi];
        const std::vector<double>& V = p->h_v[opi];
        off[2 * idx] = (long long)blob.size();
        for (int k = 0; k < r; ++k)
          for (int i = 0; i < nn; ++i) blob.push_back(U[(size_t)sg[i] * r + k]);           // U_t^T
        off[2 * idx + 1] = (long long)blob.size();
        for (int k = 0; k < r; ++k)
          for (int j = 0; j < nn; ++j) blob.push_back(V[(size_t)sg[j] * r + k]);           // V_t^T
      }
    }
    dfree(p->d_abl_ops); dfree(p->d_abl_off); dfree(p->d_abl_rank);
    p->d_abl_ops = nullptr; p->d_abl_off = nullptr; p->d_abl_rank = nullptr;
    p->abl_variant = -1;
    BBFMM_HIP_TRY(dmalloc(&p->d_abl_ops, blob.size(), nullptr));
    BBFMM_HIP_TRY(dmalloc(&p->d_abl_off, off.size(), nullptr));
    BBFMM_HIP_TRY(dmalloc(&p->d_abl_rank, rank.size(), nullptr));
    BBFMM_HIP_TRY(hipMemcpy(p->d_abl_ops, blob.data(), blob.size() * sizeof(double), hipMemcpyHostToDevice));
    BBFMM_HIP_TRY(hipMemcpy(p->d_abl_off, off.data(), off.size() * sizeof(long long), hipMemcpyHostToDevice));
    BBFMM_HIP_TRY(hipMemcpy(p->d_abl_rank, rank.data(), rank.size() * sizeof(int), hipMemcpyHostToDevice));
    p->abl_variant = variant;
    p->abl_set = set;
  }
  (void)np;
  AblationArgs a;
  a.W = d_w; a.F = d_f; a.level = level; a.scale = p->scale_of_level[level];
  a.ops = p->d_abl_ops; a.op_off = p->d_abl_off; a.op_rank = p->d_abl_rank;
  a.tab = p->d_tab; a.sig = p->d_sig; a.variant = variant; a.nrhs = nrhs;
  BBFMM_HIP_TRY(launch_m2l_unblocked(L, a, s));
  return end_call(p, s, BBFMM_OK);
}

bbfmm_status bbfmm_debug_tree_order(const bbfmm_tree* t, int32_t* d_perm, int32_t* d_leaf_start,
                                    void* stream) {
  if (!t || !d_perm || !d_leaf_start) return fail(BBFMM_EINVAL, "null argument");
  if (t->adaptive) return fail(BBFMM_EUNSUPPORTED, "uniform trees only");
  hipStream_t s = (hipStream_t)stream;
  BBFMM_HIP_TRY(hipMemcpyAsync(d_perm, t->perm, t->n * sizeof(int), hipMemcpyDeviceToDevice, s));
  BBFMM_HIP_TRY(hipMemcpyAsync(d_leaf_start, t->leaf_start, ((1LL << (3 * t->depth)) + 1) * sizeof(int),
                               hipMemcpyDeviceToDevice, s));
  return BBFMM_OK;
}

bbfmm_status bbfmm_adaptive_info_of(const bbfmm_tree* t, bbfmm_adaptive_info* out) {
  if (!t || !out) return fail(BBFMM_EINVAL, "null argument");
  if (!t->adaptive) return fail(BBFMM_EINVAL, "not an adaptive tree");
  const AdaptiveTopology& T = t->topo;
  std::memset(out, 0, sizeof(*out));
  out->n_levels = T.nlevels;
  out->n_nodes = (int32_t)T.key.size();
  out->n_leaves = (int32_t)T.leaves.size();
  out->n_u = (int64_t)T.u_idx.size();
  out->n_w = (int64_t)T.w_idx.size();
  out->n_x_nodes = (int64_t)T.x_node.size();
  out->n_x = (int64_t)T.x_idx.size();
  out->n_m2l_targets = (int64_t)T.m2l_tgt.size();
  out->v_pairs = T.v_pairs;
  out->u_point_pairs = T.u_pairs;
  out->w_pairs = T.w_pairs;
  return BBFMM_OK;
}

bbfmm_status bbfmm_adaptive_array(const bbfmm_tree* t, int32_t which, int64_t* out) {
  if (!t || !out) return fail(BBFMM_EINVAL, "null argument");
  if (!t->adaptive) return fail(BBFMM_EINVAL, "not an adaptive tree");
  const AdaptiveTopology& T = t->topo;
  auto put = [&](const auto& v) {
    for (size_t i = 0; i < v.size(); ++i) out[i] = (int64_t)v[i];
    return BBFMM_OK;
  };
  switch (which) {
    case 0: return put(T.level_off);
    case 1: return put(T.key);
    case 2: return put(T.level);
    case 3: return put(T.start);
    case 4: return put(T.end);
    case 5: return put(T.leaf);
    case 6: return put(T.child_begin);
    case 7: return put(T.child_end);
    case 8: return put(T.leaves);
    case 9: return put(T.u_off);
    case 10: return put(T.u_idx);
    case 11: return put(T.w_off);
    case 12: return put(T.w_idx);
    case 13: return put(T.x_node);
    case 14: return put(T.x_off);
    case 15: return put(T.x_idx);
    case 16: return put(T.m2l_tgt);
    case 17: return put(T.m2l_off);
    case 18: return put(T.vsrc);
    case 19: {
      if (t->xs == nullptr) return put(t->host_perm);
      std::vector<int> perm(t->n);
      BBFMM_HIP_TRY(hipMemcpy(perm.data(), t->perm, t->n * sizeof(int), hipMemcpyDeviceToHost));
      return put(perm);
    }
    default: return fail(BBFMM_EINVAL, "unknown array");
  }
}

bbfmm_status bbfmm_host_adaptive_tree(const double* points, int64_t n, int32_t max_leaf_points,
                                      const double root_lo[3], double root_width, bbfmm_tree** out) {
  if (!out) return fail(BBFMM_EINVAL, "out is null");
  *out = nullptr;
  if (!points) return fail(BBFMM_EINVAL, "null points");
  if (n < 1 || n > 0x7fffffffLL) return fail(BBFMM_EINVAL, "n must be in [1, 2^31 - 1]");
  if (max_leaf_points < 1) return fail(BBFMM_EINVAL, "max_leaf_points must be >= 1");
  if (root_width > 0 && !root_lo) return fail(BBFMM_EINVAL, "root_lo is null");
  double lo[3], hi[3];
  for (int r = 0; r < 3; ++r) {
    lo[r] = points[r];
    hi[r] = points[r];
  }
  for (long long i = 0; i < n; ++i)
    for (int r = 0; r < 3; ++r) {
      const double x = points[3 * i + r];
      if (!std::isfinite(x)) return fail(BBFMM_EINVAL, "points contain non-finite coordinates");
      lo[r] = std::min(lo[r], x);
      hi[r] = std::max(hi[r], x);
    }
  std::unique_ptr<bbfmm_tree> t(new (std::nothrow) bbfmm_tree());
  if (!t) return fail(BBFMM_ENOMEM, "host allocation");
  const double zero[3] = {0, 0, 0};
  const bbfmm_status st = root_of(lo, hi, root_lo ? root_lo : zero, root_width, t.get());
  if (st != BBFMM_OK) return st;
  t->n = n;
  t->adaptive = true;
  t->max_leaf_points = max_leaf_points;
  std::vector<int> grp;
  const std::vector<int> tab = octant_tables(&grp);
  try {
    host_adaptive_build(points, n, max_leaf_points, t->lo, t->width, tab.data(), t->topo, t->host_perm);
  } catch (const std::bad_alloc&) {
    return fail(BBFMM_ENOMEM, "host adaptive tree: host memory exhausted");
  }
  t->depth = t->topo.nlevels - 1;
  *out = t.release();
  return BBFMM_OK;
}

bbfmm_status bbfmm_host_symmetry(int32_t order, const int32_t t[3], int32_t* out_t16,
                                 int32_t* out_p, int32_t* out_sigma) {
  if (order < 2 || order > kMaxOrder) return fail(BBFMM_EUNSUPPORTED, "order must be in [2, 9]");
  const auto& reps = representatives();
  if (out_t16)
    for (int q = 0; q < kNumSym; ++q)
      for (int r = 0; r < 3; ++r) out_t16[q * 3 + r] = reps[q][r];
  if (t) {
    int linf = 0;
    for (int r = 0; r < 3; ++r) {
      if (t[r] < -3 || t[r] > 3) return fail(BBFMM_EINVAL, "|t_i| must be <= 3");
      linf = std::max(linf, std::abs(t[r]));
    }
    if (linf < 2) return fail(BBFMM_EINVAL, "t is a near-field vector");
    const int tt[3] = {t[0], t[1], t[2]};
    const SymInfo si = symmetry_of(tt);
    if (out_p) *out_p = si.p;
    if (out_sigma) sigma_table(order, si.perm_id, out_sigma);
  }
  return BBFMM_OK;
}

bbfmm_status bbfmm_host_operator(int32_t kernel, double c, int32_t order, double width, int32_t p,
                                 double svd_eps, int32_t compressor, double* out_k, double* out_u,
                                 double* out_v, int32_t* out_rank) {
  if (!valid_kernel(kernel)) return fail(BBFMM_EINVAL, "unknown kernel");
  if (order < 2 || order > kMaxOrder) return fail(BBFMM_EUNSUPPORTED, "order must be in [2, 9]");
  if (p < 0 || p >= kNumSym) return fail(BBFMM_EINVAL, "p must be in [0, 16)");
  if (!(width > 0)) return fail(BBFMM_EINVAL, "width must be > 0");
  if (compressor != BBFMM_COMPRESS_SVD && compressor != BBFMM_COMPRESS_ACA)
    return fail(BBFMM_EINVAL, "unknown compressor");
  const int nn = order * order * order;
  std::vector<double> K((size_t)nn * nn);
  m2l_operator(kernel, c, order, width, p, K.data());
  if (out_k) std::memcpy(out_k, K.data(), K.size() * sizeof(double));
  if (svd_eps > 0) {
    std::vector<double> U, V;
    const int r = compress_operator(K.data(), order, p, svd_eps, compressor, U, V);
    if (out_rank) *out_rank = r;
    if (out_u) std::memcpy(out_u, U.data(), U.size() * sizeof(double));
    if (out_v) std::memcpy(out_v, V.data(), V.size() * sizeof(double));
  } else if (out_rank) {
    *out_rank = nn;
  }
  return BBFMM_OK;
}

bbfmm_status bbfmm_host_sa_operator(int32_t kernel, double c, int32_t order, double width, double svd_eps,
                                    int32_t recompress, const int32_t t[3], double* out_u, double* out_v,
                                    int32_t* out_rank_t, int32_t* out_r) {
  if (!valid_kernel(kernel)) return fail(BBFMM_EINVAL, "unknown kernel");
  if (order < 2 || order > kMaxOrder) return fail(BBFMM_EUNSUPPORTED, "order must be in [2, 9]");
  if (!(width > 0) || !(svd_eps > 0) || !t) return fail(BBFMM_EINVAL, "width and svd_eps must be > 0, t non-null");
  if (std::max({std::abs(t[0]), std::abs(t[1]), std::abs(t[2])}) < 2 ||
      std::max({std::abs(t[0]), std::abs(t[1]), std::abs(t[2])}) > 3)
    return fail(BBFMM_EINVAL, "t is not a far-field transfer vector");
  SAOperators op;
  sa_operators(kernel, c, order, width, svd_eps, recompress != 0, op);
  const int n = op.n, r = op.r;
  const int code = (3 - t[0]) | (3 - t[1]) << 3 | (3 - t[2]) << 6;   // d = -t
  const int rt = op.rank[code];
  if (out_r) *out_r = r;
  if (out_rank_t) *out_rank_t = rt;
  // full-space factors: U_t = U C_t, V_t = U (core kept) or U_t = U Ubar, V_t = U Vbar
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < rt; ++q) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < r; ++k) {
        const double uik = op.u[(size_t)i * r + k];
        if (rt == r) {
          a += uik * op.core[code][(size_t)k * r + q];
          b = op.u[(size_t)i * r + q];
        } else {
          a += uik * op.ubar[code][(size_t)k * rt + q];
          b += uik * op.vbar[code][(size_t)k * rt + q];
        }
      }
      if (out_u) out_u[(size_t)i * rt + q] = a;
      if (out_v) out_v[(size_t)i * rt + q] = b;
    }
  return BBFMM_OK;
}

bbfmm_status bbfmm_host_singular_values(const double* a, int32_t m, int32_t n, double* out_s) {
  if (!a || !out_s) return fail(BBFMM_EINVAL, "null argument");
  if (n < 1 || m < n) return fail(BBFMM_EINVAL, "need m >= n >= 1");
  std::vector<double> U((size_t)m * n), V((size_t)n * n);
  jacobi_svd(a, m, n, U.data(), out_s, V.data());
  return BBFMM_OK;
}

}  // extern "C"
