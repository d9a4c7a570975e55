// lme_host.cpp -- host side of the C ABI declared in include/lme.h.
//
// Validation, operator pre-fold, batch planning and kernel launches.  Every
// argument is checked before the first HIP call, so malformed input is
// rejected even on a machine without a GPU.
//
// Pre-fold (Eq. (master_equation), hbar = 1):  L y = A y + y A^+ +
// sum_k C_k y C_k^+ with A = -i H0 - 1/2 sum_k C_k^+ C_k + sum_j u_j (-i H_j).
// A, -i H_j and C_k are stored as diagonal + ELL tables (lme_internal.h);
// their conjugate transposes give the adjoint L^+.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <queue>
#include <memory>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lme.h"
#include "lme_internal.h"

using cd = std::complex<double>;
using lme::InstDesc;
using lme::PackDesc;

extern "C" int lme_internal_rk4_configs(int *T, int *EPT, int cap);
extern "C" int lme_internal_pack_lds_bytes(int n, int m, int blob_bytes, int nb);
extern "C" int lme_internal_blob_stride(int blob_bytes);
extern "C" int lme_internal_lane_fits(int wo, int nb, int wb, int nc, int wc);
extern "C" hipError_t lme_internal_launch_rk4_lane(const lme::Rk4Args *a, int n_packs, int lds,
                                                   hipStream_t s);
extern "C" hipError_t lme_internal_launch_rk4(int T, int EPT, const lme::Rk4Args *a,
                                              int n_packs, int lds, hipStream_t s);
extern "C" hipError_t lme_internal_launch_rk4_colown(int cfg, int herm, int wo, int nc, int nb,
                                                     int re,
                                                     const lme::Rk4Args *a, int n_packs,
                                                     int lds, hipStream_t s);
extern "C" int lme_internal_colown_has_shape(int wo, int nc, int nb);
extern "C" int lme_internal_dp5_epts(int *ept, int cap);
extern "C" hipError_t lme_internal_launch_grad(int T, int EPT, int nq, const lme::GradArgs *a,
                                               int n_packs, int lds, hipStream_t s);
extern "C" hipError_t lme_internal_launch_grad_col(int T, int EPT, int wo, int nc,
                                                   const lme::GradArgs *a, int n_packs, int lds,
                                                   hipStream_t s);
extern "C" int lme_internal_dp5_extra_lds(int m);
extern "C" hipError_t lme_internal_launch_dp5_col(int EPT, int wo, int nc, int nb, int re,
                                                  const lme::Dp5Args *a, int n_packs, int lds,
                                                  hipStream_t s);
extern "C" hipError_t lme_internal_launch_dp5(int EPT, const lme::Dp5Args *a, int n_packs,
                                              int lds, hipStream_t s);
extern "C" hipError_t lme_internal_launch_apply_global(const lme::ApplyGArgs *a, hipStream_t s);
extern "C" hipError_t lme_internal_launch_apply_rows(int R, int re, const lme::ApplyGArgs *a,
                                                    int lds, hipStream_t s);
extern "C" hipError_t lme_internal_launch_superop(const lme::SuperArgs *a, hipStream_t s);
extern "C" hipError_t lme_internal_sdp_rows_prepare(int re, int lds);
extern "C" hipError_t lme_internal_launch_sdp_rows(int s, int re, const lme::StreamArgs *a,
                                                   int lds, hipStream_t st);
extern "C" hipError_t lme_internal_launch_sdp(int which, int arg, const lme::StreamArgs *a,
                                              hipStream_t s);
extern "C" hipError_t lme_internal_launch_apply_pipe(int wo, int nc, int nb, int re,
                                                     const lme::PipeArgs *a, int grid,
                                                     hipStream_t s);
extern "C" hipError_t lme_internal_launch_apply_col(int T, int wo, int nc, int nb, int re,
                                                    const lme::ApplyArgs *a, int n_packs,
                                                    int lds, hipStream_t s);
extern "C" hipError_t lme_internal_launch_apply_shape(int wo, int nc, int nb, int re,
                                                      const lme::ApplyArgs *a, int n_packs,
                                                      int lds, hipStream_t s);
extern "C" hipError_t lme_internal_noalloc_scratch(void **ptr, size_t *bytes);
extern "C" hipError_t lme_internal_launch_apply_lds(const lme::ApplyArgs *a, int n_packs,
                                                    int lds, hipStream_t s);

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

static int hip_fail(hipError_t e, const char *what) {
  return fail(LME_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// small host sparse matrix (rows of (col, value), sorted, merged)
// ---------------------------------------------------------------------------
struct Sparse {
  int n = 0;
  std::vector<std::vector<std::pair<int, cd>>> rows;

  explicit Sparse(int n_ = 0) : n(n_), rows(n_) {}
  void add(int i, int j, cd v) { rows[i].emplace_back(j, v); }
  void finalize() {
    for (auto &r : rows) {
      std::sort(r.begin(), r.end(),
                [](const std::pair<int, cd> &a, const std::pair<int, cd> &b) {
                  return a.first < b.first;
                });
      std::vector<std::pair<int, cd>> m;
      for (auto &e : r) {
        if (!m.empty() && m.back().first == e.first)
          m.back().second += e.second;
        else
          m.push_back(e);
      }
      r.clear();
      for (auto &e : m)
        if (e.second != cd(0.0, 0.0)) r.push_back(e);
    }
  }
  Sparse dagger() const {
    Sparse t(n);
    for (int i = 0; i < n; ++i)
      for (auto &e : rows[i]) t.add(e.first, i, std::conj(e.second));
    t.finalize();
    return t;
  }
  void axpy(cd a, const Sparse &B) {  // this += a * B
    for (int i = 0; i < n; ++i)
      for (auto &e : B.rows[i]) add(i, e.first, a * e.second);
  }
  int width_offdiag() const {
    int w = 0;
    for (int i = 0; i < n; ++i) {
      int c = 0;
      for (auto &e : rows[i]) c += (e.first != i);
      w = std::max(w, c);
    }
    return w;
  }
  int width() const {
    int w = 0;
    for (auto &r : rows) w = std::max(w, (int)r.size());
    return w;
  }
};

// C^+ C: (C^+ C)_il = sum_r conj(C_ri) C_rl
static Sparse dag_times_self(const Sparse &C) {
  Sparse out(C.n);
  for (int r = 0; r < C.n; ++r)
    for (auto &a : C.rows[r])
      for (auto &b : C.rows[r]) out.add(a.first, b.first, std::conj(a.second) * b.second);
  out.finalize();
  return out;
}

static int check_csr(const lme_csr *m, int n, const char *what, int b, Sparse *out) {
  if (!m) return fail(LME_EINVAL, "instance %d: %s is NULL", b, what);
  if (m->n != n) return fail(LME_EINVAL, "instance %d: %s has n=%d, expected %d", b, what, m->n, n);
  if (m->nnz < 0 || !m->row_ptr || (m->nnz > 0 && (!m->col || !m->val)))
    return fail(LME_EINVAL, "instance %d: %s has missing arrays", b, what);
  if (m->row_ptr[0] != 0 || m->row_ptr[n] != m->nnz)
    return fail(LME_EINVAL, "instance %d: %s row_ptr does not span [0, nnz]", b, what);
  Sparse s(n);
  for (int i = 0; i < n; ++i) {
    if (m->row_ptr[i + 1] < m->row_ptr[i])
      return fail(LME_EINVAL, "instance %d: %s row_ptr decreases at row %d", b, what, i);
    for (int p = m->row_ptr[i]; p < m->row_ptr[i + 1]; ++p) {
      const int c = m->col[p];
      if (c < 0 || c >= n)
        return fail(LME_EINVAL, "instance %d: %s column %d out of range", b, what, c);
      const double re = m->val[2 * p], im = m->val[2 * p + 1];
      if (!std::isfinite(re) || !std::isfinite(im))
        return fail(LME_EINVAL, "instance %d: %s has a non-finite value", b, what);
      s.add(i, c, cd(re, im));
    }
  }
  s.finalize();
  *out = std::move(s);
  return LME_OK;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  int upload(const void *src, size_t n, const char *what) {
    release();
    if (n == 0) return LME_OK;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      return e == hipErrorOutOfMemory ? fail(LME_ENOMEM, "hipMalloc(%s, %zu B) failed", what, n)
                                      : hip_fail(e, what);
    }
    bytes = n;
    e = hipMemcpy(p, src, n, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, what);
    return LME_OK;
  }
};

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------
struct Plan {
  int T = 0, EPT = 0, adjoint = 0, cap = 0, column = 0, dp = 0, lds_budget = 0;
  bool uploaded = false;   // d_packs / d_order hold the tables
  std::vector<PackDesc> packs;
  std::vector<int32_t> order;
  int max_lds = 0;
  DevBuf d_packs, d_order;
};

struct lme_ctx {
  int32_t n_inst = 0, n_ctrl = 0, n_e = 0, n_seg = 0;
  std::vector<double> edges;
  std::vector<InstDesc> inst;
  std::vector<int64_t> offsets;
  std::vector<int32_t> dims;
  int64_t state_elems = 0;
  int device = 0;
  int lds_limit = 0;
  // host copies of the pools, uploaded on first device use
  std::vector<uint8_t> ops, adj, eops;
  std::vector<double> u_default;
  bool on_device = false;
  DevBuf d_inst, d_ops, d_adj, d_eops, d_u;
  std::vector<Plan *> plans;
  // step tables of the last evolve call (content-cached)
  std::vector<int32_t> steps_key;
  DevBuf d_steps;
  // adaptive stepping: stop tables (content-cached) and stage derivatives
  std::vector<double> stops_key;
  DevBuf d_stops;
  DevBuf d_kbuf;
  // gradient: checkpoints and one interval of stage inputs
  DevBuf d_ckpt;
  // streamed kernels: element tiles (per instance; packed-buffer chunks)
  std::vector<lme::Tile> tiles;
  DevBuf d_tiles, d_ptiles, d_rtiles;
  int32_t n_ptiles = 0;
  // row-block application: tiles of rtile_R rows (0: not built, -1: the
  // batch has an instance outside 128 <= n <= 1024)
  int32_t n_rtiles = 0, rtile_R = 0, rtile_lds = 0;
  // streamed steppers: > 0 when their tiles are 16-row blocks (the LDS of
  // the row-block stage kernel)
  int32_t srows_lds = 0;
  // superoperator form (assembled on first use from the folded operators)
  std::vector<Sparse> A_host;
  std::vector<std::vector<Sparse>> C_host;
  DevBuf d_sd, d_scol, d_sval;
  int apply_cap = 4096;   // elements per pack of the LDS-staged application
  int apply_lds_kb = 0;   // LDS budget per column-application workgroup (0: device)
  int apply_block = 1024; // threads per column-application workgroup
  int apply_path = 0;     // column application: 0 pipelined tiles, 1 packs
  // pipelined application: row records in HBM and the tile list
  int pipe_state = 0;     // 0 not built, 1 ready, -1 not applicable
  int32_t n_pipe = 0, pipe_grid = 0;
  DevBuf d_recs, d_pt;
  // streamed steppers: workspace, per-instance tile ranges, capture stream and
  // the instantiated one-step graph (re-captured when the arguments change)
  DevBuf d_sws, d_tile_rng;
  int32_t *h_active = nullptr;   // pinned
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<uint8_t> gkey;
  lme_tuning tuning = {0, 0, 0, 0, 0.0, 0.0};
  // lme_evolve_noalloc: host image of the tables it copies into the scratch
  // array (kept until the next such call on this handle)
  std::vector<uint8_t> na_host;
  // closed-form amplitudes (lme_set_coeff_fn): [n_inst][n_ctrl][7], empty =
  // piecewise-constant segments; d_fnu holds u(t) of the last lme_apply
  std::vector<double> fn;
  DevBuf d_fn, d_fnu;
  std::vector<double> fnu_key;
  // two-time correlations: replicated batch and workspace (CorrCache)
  void *corr = nullptr;
  void (*corr_free)(void *) = nullptr;
  ~lme_ctx() {
    if (corr && corr_free) corr_free(corr);
    for (Plan *p : plans) delete p;
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (gstream) (void)hipStreamDestroy(gstream);
    if (h_active) (void)hipHostFree(h_active);
  }
};

// ---------------------------------------------------------------------------
// op blobs
// ---------------------------------------------------------------------------
struct Ell {
  std::vector<cd> val;     // [w][n]
  std::vector<int32_t> col;
};

static Ell to_ell(const Sparse &S, int w, bool offdiag_only) {
  Ell e;
  const int n = S.n;
  e.val.assign((size_t)w * n, cd(0.0, 0.0));
  e.col.resize((size_t)w * n);
  for (int i = 0; i < n; ++i) {
    int slot = 0;
    for (int s = 0; s < w; ++s) e.col[(size_t)s * n + i] = i;
    for (auto &x : S.rows[i]) {
      if (offdiag_only && x.first == i) continue;
      e.val[(size_t)slot * n + i] = x.second;
      e.col[(size_t)slot * n + i] = x.first;
      ++slot;
    }
  }
  return e;
}

static std::vector<cd> diag_of(const Sparse &S) {
  std::vector<cd> d(S.n, cd(0.0, 0.0));
  for (int i = 0; i < S.n; ++i)
    for (auto &x : S.rows[i])
      if (x.first == i) d[i] = x.second;
  return d;
}

// (memcpy with a null source is undefined even for zero bytes: an empty
// table, e.g. the off-diagonal part of a diagonal operator, copies nothing)
static void put_cd(std::vector<uint8_t> &blob, int off, const std::vector<cd> &v) {
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(cd));
}
static void put_i32(std::vector<uint8_t> &blob, int off, const std::vector<int32_t> &v) {
  if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(int32_t));
}

// Blob of (A, {B_j}, {C_k}) with A, B_j already folded.
static std::vector<uint8_t> make_blob(const Sparse &A, const std::vector<Sparse> &B,
                                      const std::vector<Sparse> &J, lme::Signature *sig) {
  const int n = A.n;
  int wo = A.width_offdiag(), wb = 0, wc = 0;
  for (auto &b : B) wb = std::max(wb, b.width_offdiag());
  for (auto &c : J) wc = std::max(wc, c.width());
  sig->n = n;
  sig->wo = wo;
  sig->nb = (int)B.size();
  sig->wb = wb;
  sig->nc = (int)J.size();
  sig->wc = wc;
  const lme::BlobLayout L = lme::blob_layout(n, wo, sig->nb, wb, sig->nc, wc);
  std::vector<uint8_t> blob((size_t)L.bytes, 0);
  put_cd(blob, L.offD, diag_of(A));
  Ell o = to_ell(A, wo, true);
  put_cd(blob, L.offOval, o.val);
  put_i32(blob, L.offOcol, o.col);
  for (int k = 0; k < sig->nc; ++k) {
    Ell e = to_ell(J[k], wc, false);
    put_cd(blob, L.offJval + 16 * k * wc * n, e.val);
    put_i32(blob, L.offJcol + 4 * k * wc * n, e.col);
  }
  for (int q = 0; q < sig->nb; ++q) {
    put_cd(blob, L.offDB + 16 * q * n, diag_of(B[q]));
    Ell e = to_ell(B[q], wb, true);
    put_cd(blob, L.offOBval + 16 * q * wb * n, e.val);
    put_i32(blob, L.offOBcol + 4 * q * wb * n, e.col);
  }
  return blob;
}

// ---------------------------------------------------------------------------
// create / destroy / layout
// ---------------------------------------------------------------------------
extern "C" void lme_default_options(lme_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof *opt);
  opt->method = LME_RK4;
  opt->path = LME_PATH_AUTO;
  opt->rtol = 1e-6;
  opt->atol = 1e-9;
  opt->max_steps = 10000000;
}

extern "C" const char *lme_last_error(void) { return g_err.c_str(); }

static int ensure_device(lme_ctx *h);

static int create_impl(int32_t n_inst, const lme_instance *inst, int32_t n_ctrl, int32_t n_e,
                       const lme_segments *seg, const double *u_host, lme_handle *out) {
  if (!out) return fail(LME_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_inst < 1 || !inst) return fail(LME_EINVAL, "n_inst must be >= 1 with a valid array");
  if (n_ctrl < 0 || n_e < 0) return fail(LME_EINVAL, "n_ctrl and n_e must be >= 0");
  if (n_ctrl > lme::kMaxWidth) return fail(LME_ENOTSUP, "at most %d control terms", lme::kMaxWidth);
  int32_t n_seg = 0;
  std::vector<double> edges;
  if (seg && seg->n_seg > 0) {
    if (!seg->edges) return fail(LME_EINVAL, "segments: edges is NULL");
    n_seg = seg->n_seg;
    edges.assign(seg->edges, seg->edges + n_seg + 1);
    for (int q = 0; q <= n_seg; ++q)
      if (!std::isfinite(edges[q])) return fail(LME_EINVAL, "segments: non-finite edge");
    for (int q = 0; q < n_seg; ++q)
      if (!(edges[q + 1] > edges[q])) return fail(LME_EINVAL, "segments: edges not increasing");
  } else if (seg && seg->n_seg < 0) {
    return fail(LME_EINVAL, "segments: n_seg < 0");
  }
  if (u_host && n_ctrl > 0 && n_seg > 0)
    for (int64_t i = 0; i < (int64_t)n_inst * n_ctrl * n_seg; ++i)
      if (!std::isfinite(u_host[i])) return fail(LME_EINVAL, "u_host has a non-finite value");

  auto *h = new (std::nothrow) lme_ctx;
  if (!h) return fail(LME_ENOMEM, "out of host memory");
  std::unique_ptr<lme_ctx> guard(h);
  h->n_inst = n_inst;
  h->n_ctrl = n_ctrl;
  h->n_e = n_e;
  h->n_seg = n_seg;
  h->edges = edges;
  h->inst.resize(n_inst);
  h->offsets.resize(n_inst);
  h->dims.resize(n_inst);

  std::vector<uint8_t> ops, adj, eops;
  for (int b = 0; b < n_inst; ++b) {
    const lme_instance &I = inst[b];
    if (!I.H0) return fail(LME_EINVAL, "instance %d: H0 is NULL", b);
    const int n = I.H0->n;
    if (n < 1) return fail(LME_EINVAL, "instance %d: n must be >= 1", b);
    if (n > lme::kMaxDim) return fail(LME_ENOTSUP, "instance %d: n=%d exceeds %d", b, n, lme::kMaxDim);
    if (I.n_c < 0 || (I.n_c > 0 && !I.C)) return fail(LME_EINVAL, "instance %d: bad collapse list", b);
    if (n_ctrl > 0 && !I.H_ctrl) return fail(LME_EINVAL, "instance %d: H_ctrl is NULL", b);
    if (n_e > 0 && !I.E) return fail(LME_EINVAL, "instance %d: E is NULL", b);
    Sparse H, tmp;
    int rc = check_csr(I.H0, n, "H0", b, &H);
    if (rc) return rc;
    std::vector<Sparse> Hc(n_ctrl), C(I.n_c), E(n_e);
    for (int j = 0; j < n_ctrl; ++j)
      if ((rc = check_csr(&I.H_ctrl[j], n, "H_ctrl", b, &Hc[j]))) return rc;
    for (int k = 0; k < I.n_c; ++k)
      if ((rc = check_csr(&I.C[k], n, "C", b, &C[k]))) return rc;
    for (int m = 0; m < n_e; ++m)
      if ((rc = check_csr(&I.E[m], n, "E", b, &E[m]))) return rc;

    // A0 = -i H0 - 1/2 sum_k C_k^+ C_k ;  B_j = -i H_j
    Sparse A(n);
    A.axpy(cd(0.0, -1.0), H);
    for (auto &c : C) A.axpy(cd(-0.5, 0.0), dag_times_self(c));
    A.finalize();
    std::vector<Sparse> B(n_ctrl, Sparse(n)), Bt, Ct;
    for (int j = 0; j < n_ctrl; ++j) {
      B[j].axpy(cd(0.0, -1.0), Hc[j]);
      B[j].finalize();
      Bt.push_back(B[j].dagger());
    }
    for (auto &c : C) Ct.push_back(c.dagger());
    Sparse At = A.dagger();
    for (auto *S : {&A, &At}) {
      if (S->width_offdiag() > lme::kMaxWidth)
        return fail(LME_ENOTSUP, "instance %d: operator row wider than %d", b, lme::kMaxWidth);
    }
    for (auto &c : C)
      if (c.width() > lme::kMaxWidth || c.dagger().width() > lme::kMaxWidth)
        return fail(LME_ENOTSUP, "instance %d: collapse operator row wider than %d", b, lme::kMaxWidth);
    for (auto &x : B)
      if (x.width_offdiag() > lme::kMaxWidth || x.dagger().width_offdiag() > lme::kMaxWidth)
        return fail(LME_ENOTSUP, "instance %d: control operator row wider than %d", b, lme::kMaxWidth);

    h->A_host.push_back(A);
    h->C_host.push_back(C);
    InstDesc &d = h->inst[b];
    d.flags = 0;
    {
      bool jr = true, oi = true;
      for (auto &c : C)
        for (auto &row : c.rows)
          for (auto &e : row) jr = jr && e.second.imag() == 0.0;
      auto offdiag_imag = [](const Sparse &S) {
        for (int i = 0; i < S.n; ++i)
          for (auto &e : S.rows[i])
            if (e.first != i && e.second.real() != 0.0) return false;
        return true;
      };
      oi = offdiag_imag(A);
      for (auto &x : B) oi = oi && offdiag_imag(x);
      d.flags = (jr ? lme::kJumpsReal : 0) | (oi ? lme::kOffdiagImag : 0);
    }
    std::vector<uint8_t> fb = make_blob(A, B, C, &d.fwd);
    std::vector<uint8_t> ab = make_blob(At, Bt, Ct, &d.adj);
    d.n = n;
    d.fwd_bytes = (int32_t)fb.size();
    d.adj_bytes = (int32_t)ab.size();
    d.ops_off = (int64_t)ops.size();
    d.adj_off = (int64_t)adj.size();
    ops.insert(ops.end(), fb.begin(), fb.end());
    adj.insert(adj.end(), ab.begin(), ab.end());

    // expectation operators: full ELL, Ecol[m][we][n], Eval[m][we][n]
    int we = 1;
    for (auto &e : E) we = std::max(we, e.width());
    if (we > lme::kMaxWidth) return fail(LME_ENOTSUP, "instance %d: e-op row wider than %d", b, lme::kMaxWidth);
    d.we = we;
    d.eops_off = (int64_t)eops.size();
    std::vector<uint8_t> eb((size_t)lme::eops_bytes(n, we, n_e), 0);
    for (int m = 0; m < n_e; ++m) {
      Ell e = to_ell(E[m], we, false);
      std::memcpy(eb.data() + 4 * (size_t)m * we * n, e.col.data(), e.col.size() * 4);
      std::memcpy(eb.data() + lme::eops_val_offset(n, we, n_e) + 16 * (size_t)m * we * n,
                  e.val.data(), e.val.size() * 16);
    }
    eb.resize((size_t)lme::align16((int32_t)eb.size()));
    eops.insert(eops.end(), eb.begin(), eb.end());

    d.rho_off = h->state_elems;
    h->offsets[b] = h->state_elems;
    h->dims[b] = n;
    h->state_elems += (int64_t)n * n;
  }

  h->ops.swap(ops);
  h->adj.swap(adj);
  h->eops.swap(eops);
  if (n_ctrl > 0 && n_seg > 0) {
    h->u_default.assign((size_t)n_inst * n_ctrl * n_seg, 0.0);
    if (u_host) std::memcpy(h->u_default.data(), u_host, h->u_default.size() * sizeof(double));
  }
  // With a device present, bind it and upload the operator tables now (a
  // machine without one defers this to the first device call).
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) == hipSuccess && n_dev > 0) {
    const int rc = ensure_device(h);
    if (rc) return rc;
  } else {
    (void)hipGetLastError();
  }
  *out = guard.release();
  return LME_OK;
}

extern "C" int lme_create_batch(int32_t n_inst, const lme_instance *inst, int32_t n_ctrl,
                                int32_t n_e, const lme_segments *seg, const double *u_host,
                                lme_handle *out) {
  try {
    return create_impl(n_inst, inst, n_ctrl, n_e, seg, u_host, out);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

extern "C" int lme_create(const lme_csr *H0, int32_t n_ctrl, const lme_csr *H_ctrl,
                          const lme_segments *seg, const double *u_host, int32_t n_c,
                          const lme_csr *C, int32_t n_e, const lme_csr *E, lme_handle *out) {
  lme_instance I;
  I.H0 = H0;
  I.H_ctrl = H_ctrl;
  I.n_c = n_c;
  I.C = C;
  I.E = E;
  return lme_create_batch(1, &I, n_ctrl, n_e, seg, u_host, out);
}

extern "C" void lme_destroy(lme_handle h) { delete h; }

extern "C" int lme_set_coeff_fn(lme_handle h, const double *fn_host) {
  try {
    if (!h) return fail(LME_EINVAL, "handle is NULL");
    if (!fn_host) {
      h->fn.clear();
      h->d_fn.release();
      h->d_fnu.release();
      h->fnu_key.clear();
      return LME_OK;
    }
    if (h->n_ctrl < 1) return fail(LME_EINVAL, "the batch has no control terms");
    const size_t cnt = (size_t)h->n_inst * h->n_ctrl * 7;
    for (size_t i = 0; i < cnt; ++i)
      if (!std::isfinite(fn_host[i])) return fail(LME_EINVAL, "fn has a non-finite value");
    std::vector<double> fn(fn_host, fn_host + cnt);
    if (h->on_device) {
      int rc = ensure_device(h);
      if (rc) return rc;
      if ((rc = h->d_fn.upload(fn.data(), cnt * sizeof(double), "closed-form amplitudes")))
        return rc;
    }
    h->fn.swap(fn);
    h->fnu_key.clear();
    return LME_OK;
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

extern "C" int lme_layout(lme_handle h, int32_t *n_inst, int64_t *state_elems,
                          int64_t *offsets, int32_t *dims) {
  if (!h) return fail(LME_EINVAL, "handle is NULL");
  if (n_inst) *n_inst = h->n_inst;
  if (state_elems) *state_elems = h->state_elems;
  if (offsets) std::memcpy(offsets, h->offsets.data(), h->offsets.size() * sizeof(int64_t));
  if (dims) std::memcpy(dims, h->dims.data(), h->dims.size() * sizeof(int32_t));
  return LME_OK;
}

// ---------------------------------------------------------------------------
// first device use: bind the current device and upload the operator pools
// ---------------------------------------------------------------------------
static int ensure_device(lme_ctx *h) {
  hipError_t e;
  if (h->on_device) {
    e = hipSetDevice(h->device);
    return e == hipSuccess ? LME_OK : hip_fail(e, "hipSetDevice");
  }
  e = hipGetDevice(&h->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  int lds = 0;
  e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(LDS)");
  h->lds_limit = lds;
  int rc;
  if ((rc = h->d_inst.upload(h->inst.data(), h->inst.size() * sizeof(InstDesc), "instances"))) return rc;
  if ((rc = h->d_ops.upload(h->ops.data(), h->ops.size(), "op pool"))) return rc;
  if ((rc = h->d_adj.upload(h->adj.data(), h->adj.size(), "adjoint op pool"))) return rc;
  if ((rc = h->d_eops.upload(h->eops.data(), h->eops.size(), "e-op pool"))) return rc;
  if (!h->u_default.empty() &&
      (rc = h->d_u.upload(h->u_default.data(), h->u_default.size() * sizeof(double), "controls")))
    return rc;
  if (!h->fn.empty() &&
      (rc = h->d_fn.upload(h->fn.data(), h->fn.size() * sizeof(double), "closed-form amplitudes")))
    return rc;
  h->on_device = true;
  return LME_OK;
}

// ---------------------------------------------------------------------------
// planning: group instances by operator signature, fill packs
// ---------------------------------------------------------------------------
// Row layout (column == 0): packs of up to `cap` elements.
// Column layout (column == 1): per signature group choose G (threads per
// column) and m (instances per pack) with m*n*G <= T and ceil(n/G) <= EPT,
// maximising the fraction of the workgroup's T*ept element slots in use.
// Hermitian column layout (column == 2): the same with n/2 + 1 rows per
// column.  Column application (column == 3): as column == 1.
// LDS operator data per instance: the op blob (row and column RK4 kernels),
// one record per operator row (column application, Hermitian kernel) or
// nothing (Hermitian kernel with real structure and no control terms: its
// row data lives in registers).
static int real_structure(const lme_ctx *h);

static int upload_plan(Plan *p) {
  int rc;
  if ((rc = p->d_packs.upload(p->packs.data(), p->packs.size() * sizeof(PackDesc), "packs"))) return rc;
  if ((rc = p->d_order.upload(p->order.data(), p->order.size() * sizeof(int32_t), "order"))) return rc;
  p->uploaded = true;
  return LME_OK;
}

// upload = false: the host tables only (lme_evolve_noalloc copies them into
// its scratch array); a later call with upload = true uploads a cached plan.
static int plan_packs(lme_ctx *h, int T, int EPT, int adjoint, int cap, int column, int dp,
                      Plan **out, int lds_budget = 0, bool upload = true) {
  for (Plan *p : h->plans)
    if (p->T == T && p->EPT == EPT && p->adjoint == adjoint && p->cap == cap &&
        p->column == column && p->dp == dp && p->lds_budget == lds_budget) {
      if (upload && !p->uploaded) {
        const int rc = upload_plan(p);
        if (rc) return rc;
      }
      *out = p;
      return LME_OK;
    }
  // adjoint: 0 forward blobs, 1 adjoint blobs, 2 both (gradient kernel)
  auto key = [&](const InstDesc &d) {
    const lme::Signature &s = adjoint == 1 ? d.adj : d.fwd;
    const lme::Signature &t = d.adj;
    return std::make_tuple(s.n, s.wo, s.nb, s.wb, s.nc, s.wc,
                           adjoint == 2 ? t.wo : 0, adjoint == 2 ? t.wb : 0,
                           adjoint == 2 ? t.wc : 0);
  };
  std::map<std::tuple<int, int, int, int, int, int, int, int, int>, std::vector<int32_t>> groups;
  for (int b = 0; b < h->n_inst; ++b) groups[key(h->inst[b])].push_back(b);

  std::unique_ptr<Plan> p(new Plan);
  p->T = T;
  p->EPT = EPT;
  p->adjoint = adjoint;
  p->cap = cap;
  p->column = column;
  p->dp = dp;
  p->lds_budget = lds_budget;
  // LDS of a pack of m instances (the adaptive kernel adds its step control)
  // dp: 1 adaptive kernel (step control), 2 gradient kernel (sums)
  auto pack_lds = [&](int n, int m, int blob, int nb) {
    return lme_internal_pack_lds_bytes(n, m, blob, nb) +
           (dp == 1 ? lme_internal_dp5_extra_lds(m) : dp == 2 ? lme::align16(8 * m) : 0);
  };
  for (auto &g : groups) {
    const InstDesc &d0 = h->inst[g.second[0]];
    const lme::Signature &s = adjoint == 1 ? d0.adj : d0.fwd;
    const int blob = column == 2 && lme::herm_slots(real_structure(h), s.wo, s.nc, s.nb) ? 0
                     : column >= 2 ? s.n * lme::rec_bytes(s.wo, s.nc, s.nb)
                     : adjoint == 1 ? d0.adj_bytes
                     : adjoint == 2 ? d0.fwd_bytes + d0.adj_bytes : d0.fwd_bytes;
    const int n = s.n;
    const int64_t n2 = (int64_t)n * n;
    const int cnt = (int)g.second.size();
    // m instances that fit the LDS budget; an instance larger than the
    // budget alone gets the device limit
    auto lds_fit_in = [&](int64_t m, int64_t limit) {
      // at most kMaxPack instances (the kernels encode the pack slot in 10 bits)
      m = std::min<int64_t>(m, lme::kMaxPack);
      const int64_t per_inst = 16 * n2 + blob + 16 + 8LL * s.nb + 12 +
                               (dp ? 128 : 0);  // upper bound
      m = std::min<int64_t>(m, std::max<int64_t>(0, (limit - 48) / per_inst));
      while (m > 0 && pack_lds(n, (int)m, blob, s.nb) > limit) --m;
      return (int)m;
    };
    auto lds_fit = [&](int64_t m) {
      const int64_t budget = lds_budget > 0 ? std::min<int64_t>(lds_budget, h->lds_limit)
                                            : h->lds_limit;
      const int r = lds_fit_in(m, budget);
      return (r > 0 || budget == h->lds_limit) ? r : lds_fit_in(std::min<int64_t>(m, 1), h->lds_limit);
    };
    int m_max = 0, G = 0;
    const int R = column == 2 ? n / 2 + 1 : n;  // rows per column
    if (!column) {
      m_max = lds_fit(std::max<int64_t>(1, cap / n2));  // an instance larger than cap: alone
    } else {
      double best = -1.0;
      for (int gg = (R + EPT - 1) / EPT; gg <= R && gg * n <= T; ++gg) {
        const int ept = (R + gg - 1) / gg;
        const int m = lds_fit(std::min<int64_t>(T / (gg * n), cnt));
        if (m < 1) continue;
        const double eff = (double)m * n * R / ((double)ept * T);
        if (eff > best + 1e-12) {
          best = eff;
          m_max = m;
          G = gg;
        }
      }
    }
    if (m_max < 1)
      return fail(LME_ENOTSUP, "instance of dimension %d does not fit a resident workgroup "
                  "(%s layout, %d B LDS available)", n, column ? "column" : "row", h->lds_limit);
    const int n_packs = (cnt + m_max - 1) / m_max;
    // spread the group evenly over its packs
    int done = 0;
    for (int q = 0; q < n_packs; ++q) {
      const int m = (cnt - done + (n_packs - q) - 1) / (n_packs - q);
      PackDesc pk;
      pk.first = (int32_t)p->order.size();
      pk.m = m;
      pk.n = n;
      pk.wo = s.wo;
      pk.nb = s.nb;
      pk.wb = s.wb;
      pk.nc = s.nc;
      pk.wc = s.wc;
      pk.blob_bytes = blob;
      pk.lds_bytes = pack_lds(n, m, blob, s.nb);
      pk.G = G;
      pk.ept = G > 0 ? (R + G - 1) / G : 0;
      pk.awo = d0.adj.wo;
      pk.awb = d0.adj.wb;
      pk.awc = d0.adj.wc;
      pk.fwd_bytes = d0.fwd_bytes;
      pk.blob_stride = lme_internal_blob_stride(blob);
      pk.pad_ = 0;
      for (int r = 0; r < m; ++r) p->order.push_back(g.second[done + r]);
      done += m;
      p->packs.push_back(pk);
      p->max_lds = std::max(p->max_lds, pk.lds_bytes);
    }
  }
  // longest first (the hardware hands workgroups to free CUs roughly in
  // order, so this is a longest-processing-time schedule): a column-layout
  // pack takes time in proportion to its rows per thread, a row-layout pack
  // to its elements
  auto longest_first = [&]() {
    std::stable_sort(p->packs.begin(), p->packs.end(), [](const PackDesc &a, const PackDesc &b) {
      if (a.ept != b.ept) return a.ept > b.ept;
      return (int64_t)a.m * a.n * a.n > (int64_t)b.m * b.n * b.n;
    });
  };
  longest_first();
  // Column layouts, one workgroup per CU: while the pack that finishes last
  // in that schedule holds several instances and half of them fit more
  // threads per column (fewer rows per thread), split it in two.  Packing
  // changes no result bit.
  int cus = 0;
  if (column >= 1 && column <= 2 &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
      cus > 0) {
    for (int iter = 0; iter < 4 * cus; ++iter) {
      std::priority_queue<std::pair<int64_t, int>, std::vector<std::pair<int64_t, int>>,
                          std::greater<std::pair<int64_t, int>>> free_at;
      for (int c = 0; c < cus; ++c) free_at.push({0, c});
      int64_t makespan = 0;
      int last = -1;
      for (int q = 0; q < (int)p->packs.size(); ++q) {
        auto top = free_at.top();
        free_at.pop();
        const int64_t end = top.first + p->packs[q].ept;
        if (end >= makespan) {
          makespan = end;
          last = q;
        }
        free_at.push({end, top.second});
      }
      if (last < 0) break;
      PackDesc pk = p->packs[last];
      if (pk.m < 2) break;
      const int R = column == 2 ? pk.n / 2 + 1 : pk.n;
      const int m1 = (pk.m + 1) / 2, m2 = pk.m - m1;
      const int G1 = std::min(R, T / (m1 * pk.n));
      const int ept1 = (R + G1 - 1) / G1;
      if (ept1 >= pk.ept) break;
      const int G2 = std::min(R, T / (m2 * pk.n));
      PackDesc a = pk, b = pk;
      a.m = m1;
      a.G = G1;
      a.ept = ept1;
      a.lds_bytes = pack_lds(pk.n, m1, pk.blob_bytes, pk.nb);
      b.first = pk.first + m1;
      b.m = m2;
      b.G = G2;
      b.ept = (R + G2 - 1) / G2;
      b.lds_bytes = pack_lds(pk.n, m2, pk.blob_bytes, pk.nb);
      p->packs[last] = a;
      p->packs.push_back(b);
      longest_first();
    }
    for (const PackDesc &q : p->packs) {  // what the column kernels assume
      const int R = column == 2 ? q.n / 2 + 1 : q.n;
      if (q.m < 1 || (int64_t)q.m * q.n * q.G > T || q.G > R || q.ept > EPT ||
          q.ept != (R + q.G - 1) / q.G)
        return fail(LME_EINVAL, "internal: inconsistent pack (n %d, m %d, G %d, rows %d)", q.n,
                    q.m, q.G, q.ept);
    }
  }
  if (upload) {
    const int rc = upload_plan(p.get());
    if (rc) return rc;
  }
  *out = p.get();
  h->plans.push_back(p.release());
  return LME_OK;
}

// ---------------------------------------------------------------------------
// lme_evolve_noalloc: tables and stage derivatives in the scratch array
// ---------------------------------------------------------------------------
// Scratch layout: [tables | packs | order | stage derivatives], each part
// 256-byte aligned.  The host part is assembled in h->na_host and copied with
// one hipMemcpyAsync on the caller's stream.
struct NoAlloc {
  uint8_t *base = nullptr;
  size_t cap = 0;
  size_t packs_off = 0, order_off = 0, kbuf_off = 0, total = 0;
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

static int noalloc_stage(lme_ctx *h, const void *tab, size_t tab_bytes, const Plan *plan,
                         size_t kbuf_bytes, hipStream_t s, NoAlloc *na) {
  void *p = nullptr;
  size_t cap = 0;
  hipError_t e = lme_internal_noalloc_scratch(&p, &cap);
  if (e != hipSuccess) return hip_fail(e, "scratch array address");
  na->base = static_cast<uint8_t *>(p);
  na->cap = cap;
  na->packs_off = align256(tab_bytes);
  na->order_off = align256(na->packs_off + plan->packs.size() * sizeof(PackDesc));
  const size_t host_end = na->order_off + plan->order.size() * sizeof(int32_t);
  na->kbuf_off = align256(host_end);
  na->total = na->kbuf_off + kbuf_bytes;
  if (na->total > cap)
    return fail(LME_ENOTSUP, "lme_evolve_noalloc needs %zu bytes of scratch; its array holds %zu "
                "(the adaptive stepper's stage derivatives take 112 bytes per state element)",
                na->total, cap);
  h->na_host.assign(host_end, 0);
  if (tab_bytes) std::memcpy(h->na_host.data(), tab, tab_bytes);
  std::memcpy(h->na_host.data() + na->packs_off, plan->packs.data(),
              plan->packs.size() * sizeof(PackDesc));
  std::memcpy(h->na_host.data() + na->order_off, plan->order.data(),
              plan->order.size() * sizeof(int32_t));
  e = hipMemcpyAsync(na->base, h->na_host.data(), host_end, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "copy tables into the scratch array");
  return LME_OK;
}

// ---------------------------------------------------------------------------
// time grid
// ---------------------------------------------------------------------------
static long grid_index(double t, double t0, double h) {
  const long m = std::lround((t - t0) / h);
  if (std::fabs(t - (t0 + (double)m * h)) > 1e-6 * std::fabs(h)) return -1;
  return m;
}

// Segment holding time t, or -1.
static int segment_at(const lme_ctx *h, double t) {
  if (h->n_seg == 0 || t < h->edges[0] || t >= h->edges[h->n_seg]) return -1;
  const auto it = std::upper_bound(h->edges.begin(), h->edges.end(), t);
  return (int)(it - h->edges.begin()) - 1;
}

static int check_times(int32_t n_t, const double *tlist) {
  if (n_t < 1 || !tlist) return fail(LME_EINVAL, "need n_t >= 1 output times");
  for (int k = 0; k < n_t; ++k)
    if (!std::isfinite(tlist[k])) return fail(LME_EINVAL, "tlist[%d] is not finite", k);
  for (int k = 1; k < n_t; ++k)
    if (!(tlist[k] > tlist[k - 1])) return fail(LME_EINVAL, "tlist must be strictly increasing");
  return LME_OK;
}

// Builds [seg_of_step[nsteps] | out_step[n_t]] (host only, validates the grid).
static int rk4_tables(const lme_ctx *h, int32_t n_t, const double *tlist, int32_t nsteps,
                      double hstep, std::vector<int32_t> *out) {
  std::vector<int32_t> tab((size_t)nsteps + n_t);
  const double t0 = tlist[0];
  tab[nsteps] = 0;
  for (int k = 1; k < n_t; ++k) {
    const long m = grid_index(tlist[k], t0, hstep);
    if (m < 0 || m > nsteps)
      return fail(LME_EGRID, "output time %.17g is not on the RK4 grid (h = %.17g)", tlist[k], hstep);
    tab[nsteps + k] = (int32_t)m;
  }
  if (n_t > 1 && tab[nsteps + n_t - 1] != nsteps)
    return fail(LME_EGRID, "last output time is not the end of the grid");
  const double t1 = tlist[n_t - 1];
  for (int q = 0; q <= h->n_seg && h->n_seg > 0 && h->fn.empty(); ++q) {
    const double e = h->edges[q];
    if (e > t0 && e < t1 && grid_index(e, t0, hstep) < 0)
      return fail(LME_EGRID, "control edge %.17g is not on the RK4 grid", e);
  }
  for (int st = 0; st < nsteps; ++st) tab[st] = segment_at(h, t0 + ((double)st + 0.5) * hstep);
  out->swap(tab);
  return LME_OK;
}

// Uploads the step tables unless the previous call used identical ones.
static int upload_tables(lme_ctx *h, std::vector<int32_t> &tab, hipStream_t s) {
  if (tab == h->steps_key && h->d_steps.p) return LME_OK;
  h->d_steps.release();
  hipError_t e = hipMalloc(&h->d_steps.p, tab.size() * sizeof(int32_t));
  if (e != hipSuccess) {
    h->d_steps.p = nullptr;
    return hip_fail(e, "hipMalloc(step tables)");
  }
  h->d_steps.bytes = tab.size() * sizeof(int32_t);
  e = hipMemcpyAsync(h->d_steps.p, tab.data(), h->d_steps.bytes, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "upload step tables");
  h->steps_key.swap(tab);
  return LME_OK;
}

// ---------------------------------------------------------------------------
// evolve
// ---------------------------------------------------------------------------
static int pick_rk4_config(const lme_ctx *h, int block, int *T, int *EPT, int *cap = nullptr) {
  int max_n2 = 0;
  int64_t tot = 0;
  for (auto &d : h->inst) {
    max_n2 = std::max(max_n2, d.n * d.n);
    tot += (int64_t)d.n * d.n;
  }
  int Ts[64], Es[64];
  const int nc = lme_internal_rk4_configs(Ts, Es, 64);
  int want_T = block > 0 ? block : 512;
  // small instances whose whole batch would fill fewer than two 512-thread
  // workgroups per CU: one wavefront per pack, so that every CU gets packs
  // (and the stage barriers are a single wavefront's)
  int cus = 0;
  if (block <= 0 && max_n2 <= 64 * 8 &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
      cus > 0 && tot < (int64_t)2 * 512 * cus)
    want_T = 64;
  int best = -1;
  for (int i = 0; i < nc; ++i)
    if (Ts[i] == want_T && Ts[i] * Es[i] >= max_n2 && (best < 0 || Es[i] < Es[best])) best = i;
  if (best < 0 && block <= 0)  // any block size that fits
    for (int i = 0; i < nc; ++i)
      if (Ts[i] * Es[i] >= max_n2 && (best < 0 || Ts[i] * Es[i] < Ts[best] * Es[best])) best = i;
  if (best < 0)
    return fail(LME_ENOTSUP, "largest instance (%d elements) exceeds the resident RK4 "
                "workgroup capacity for block %d", max_n2, want_T);
  *T = Ts[best];
  *EPT = Es[best];
  if (cap) {
    // one-wavefront packs: at most a quarter of the batch per CU slot (so
    // that a CU holds several latency-bound wavefronts), never below one
    // instance
    *cap = Ts[best] * Es[best];
    if (Ts[best] == 64 && cus > 0)
      *cap = (int)std::max<int64_t>(max_n2, std::min<int64_t>(*cap, tot / (4 * cus)));
  }
  return LME_OK;
}

// Can every instance use the column-owner kernels?  They need one operator
// shape across the batch (off-diagonal width of A, number of monomial collapse
// operators, at most one control term of width <= kColWB) with a compiled
// instantiation, and n < 256 (row indices are packed 8 bits apiece).
static bool column_eligible(const lme_ctx *h, int *wo, int *nc, int *nb) {
  const lme::Signature &s0 = h->inst[0].fwd;
  for (auto &d : h->inst) {
    const lme::Signature &s = d.fwd;
    if (s.wo != s0.wo || s.nc != s0.nc || s.nb != s0.nb) return false;
    if ((s.nc > 0 && s.wc != 1) || s.nb > 1 || s.wb > lme::kColWB || s.n > 255) return false;
  }
  if (!lme_internal_colown_has_shape(s0.wo, s0.nc, s0.nb)) return false;
  *wo = s0.wo;
  *nc = s0.nc;
  *nb = s0.nb;
  return true;
}

// 1 when every instance has real jump coefficients and purely imaginary
// off-diagonal entries of A and of the control terms.
static int real_structure(const lme_ctx *h) {
  for (auto &d : h->inst)
    if ((d.flags & (lme::kJumpsReal | lme::kOffdiagImag)) != (lme::kJumpsReal | lme::kOffdiagImag))
      return 0;
  return 1;
}

static bool column_fits(const lme_ctx *h, int T, int EPT, bool herm) {
  for (auto &d : h->inst) {
    const int n = d.n, R = herm ? n / 2 + 1 : n;
    if ((int64_t)n * ((R + EPT - 1) / EPT) > T) return false;
  }
  return true;
}

// Stop points of the adaptive stepper: every output time after tlist[0] and
// every control edge inside (tlist[0], tlist[n_t-1]), sorted, duplicates
// removed.  Packed as [stops (double) | out index | segment] into 8-byte
// slots: stops[n], then 2n int32.
static int dp5_tables(const lme_ctx *h, int32_t n_t, const double *tlist,
                      std::vector<double> *stops, std::vector<int32_t> *out_idx,
                      std::vector<int32_t> *seg) {
  const double t0 = tlist[0], t1 = tlist[n_t - 1];
  std::vector<double> st(tlist + 1, tlist + n_t);
  for (int q = 0; q <= h->n_seg && h->n_seg > 0; ++q)
    if (h->edges[q] > t0 && h->edges[q] < t1) st.push_back(h->edges[q]);
  std::sort(st.begin(), st.end());
  st.erase(std::unique(st.begin(), st.end()), st.end());
  out_idx->assign(st.size(), -1);
  seg->assign(st.size(), -1);
  int k = 1;
  double prev = t0;
  for (size_t i = 0; i < st.size(); ++i) {
    while (k < n_t && tlist[k] < st[i]) ++k;
    if (k < n_t && tlist[k] == st[i]) (*out_idx)[i] = k;
    (*seg)[i] = segment_at(h, 0.5 * (prev + st[i]));
    prev = st[i];
  }
  stops->swap(st);
  return LME_OK;
}

static int ensure_tiles(lme_ctx *h);

// Workspace of the streamed steppers: rho, two stage-input buffers, the
// fifth-order solution, the RK4 accumulator, seven stage derivatives, tile
// partial sums and per-instance control; plus per-instance tile ranges.
static int stream_workspace(lme_ctx *h, lme::StreamArgs *a) {
  int rc = ensure_tiles(h);
  if (rc) return rc;
  const size_t SE16 = (size_t)h->state_elems * 16;
  const size_t nt = h->tiles.size();
  const size_t ctl = lme::align16((int32_t)sizeof(lme::DpCtl)) * (size_t)h->n_inst;
  const size_t need = 12 * SE16 + 16 * nt + ctl + 256;
  if (h->d_sws.bytes < need) {
    h->d_sws.release();
    hipError_t e = hipMalloc(&h->d_sws.p, need);
    if (e != hipSuccess) {
      h->d_sws.p = nullptr;
      return fail(LME_ENOMEM, "hipMalloc(streamed workspace, %zu B) failed", need);
    }
    h->d_sws.bytes = need;
  }
  if (!h->d_tile_rng.p) {
    std::vector<int32_t> rng(2 * (size_t)h->n_inst, 0);
    for (size_t q = 0; q < nt; ++q) {
      const int b = h->tiles[q].inst;
      if (rng[2 * b + 1] == 0) rng[2 * b] = (int32_t)q;
      ++rng[2 * b + 1];
    }
    std::vector<int32_t> packed(2 * (size_t)h->n_inst);
    for (int b = 0; b < h->n_inst; ++b) {
      packed[b] = rng[2 * b];
      packed[h->n_inst + b] = rng[2 * b + 1];
    }
    if ((rc = h->d_tile_rng.upload(packed.data(), packed.size() * 4, "tile ranges"))) return rc;
  }
  if (!h->h_active) {
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&h->h_active), 16, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
  }
  uint8_t *p = static_cast<uint8_t *>(h->d_sws.p);
  a->rho = reinterpret_cast<double *>(p);
  a->yb0 = reinterpret_cast<double *>(p + SE16);
  a->yb1 = reinterpret_cast<double *>(p + 2 * SE16);
  a->y5 = reinterpret_cast<double *>(p + 3 * SE16);
  a->acc = reinterpret_cast<double *>(p + 4 * SE16);
  a->K = reinterpret_cast<double *>(p + 5 * SE16);
  a->tile_part = reinterpret_cast<double *>(p + 12 * SE16);
  a->ctl = reinterpret_cast<lme::DpCtl *>(p + 12 * SE16 + 16 * nt);
  a->n_active = reinterpret_cast<int32_t *>(p + 12 * SE16 + 16 * nt + ctl);
  a->counters = a->n_active + 4;
  a->tiles = static_cast<const lme::Tile *>(h->d_tiles.p);
  a->n_tiles = (int32_t)nt;
  a->n_inst = h->n_inst;
  a->tile_first = static_cast<const int32_t *>(h->d_tile_rng.p);
  a->tile_count = a->tile_first + h->n_inst;
  a->inst = static_cast<const InstDesc *>(h->d_inst.p);
  a->ops = static_cast<const uint8_t *>(h->d_ops.p);
  a->eops = static_cast<const uint8_t *>(h->d_eops.p);
  a->n_ctrl = h->n_ctrl;
  a->n_seg = h->n_seg;
  a->n_e = h->n_e;
  a->state_elems = h->state_elems;
  if (!h->gstream) {
    hipError_t e = hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      h->gstream = nullptr;
      return hip_fail(e, "hipStreamCreate");
    }
  }
  return LME_OK;
}

// Captures `record` (a sequence of launches on the given stream) into the
// handle's graph unless the arguments are those of the cached graph.
template <typename F>
static int cached_graph(lme_ctx *h, const void *key, size_t key_bytes, F &&record) {
  std::vector<uint8_t> k(static_cast<const uint8_t *>(key), static_cast<const uint8_t *>(key) + key_bytes);
  if (h->gexec && k == h->gkey) return LME_OK;
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  const int rc = record(h->gstream);
  e = hipStreamEndCapture(h->gstream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    h->gexec = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  h->gkey.swap(k);
  return LME_OK;
}

// Streamed Dormand-Prince: the sequence of kernels of one attempted step is
// captured once as a graph and replayed; the host reads the active count
// every kReplay replays.  Every replay makes one attempt for every active
// instance and every instance stops within max_steps attempts, so the loop
// ends after at most max_steps + 1 replays.
static int evolve_dp5_streamed(lme_ctx *h, const lme_options *opt, int32_t n_t,
                               const double *tlist, const void *rho0_dev,
                               const double *u_dev, void *expect_dev, void *states_dev,
                               void *rho_out_dev, int64_t *counts_dev, int32_t *status_dev,
                               hipStream_t s, const lme::Dp5Args &tabs) {
  lme::StreamArgs a;
  std::memset(&a, 0, sizeof a);
  int rc = stream_workspace(h, &a);
  if (rc) return rc;
  a.u = u_dev ? u_dev : static_cast<const double *>(h->d_u.p);
  a.n_t = n_t;
  a.stops = tabs.stops;
  a.stop_out = tabs.stop_out;
  a.stop_seg = tabs.stop_seg;
  a.n_stops = tabs.n_stops;
  a.t0 = tlist[0];
  a.rtol = opt->rtol;
  a.atol = opt->atol;
  a.h0 = opt->h0;
  a.h_min = opt->h_min;
  a.max_steps = opt->max_steps;
  a.states = static_cast<double *>(states_dev);
  a.expect = static_cast<double *>(expect_dev);
  a.counts = counts_dev;
  a.status = status_dev;
  const int re = real_structure(h);
  if (h->srows_lds > 0) {
    hipError_t e = lme_internal_sdp_rows_prepare(re, h->srows_lds);
    if (e != hipSuccess) return hip_fail(e, "set up the row-block stage kernel");
  }
  auto L = [&](int which, int arg, hipStream_t st) -> int {
    hipError_t e = which == 0 && h->srows_lds > 0
                       ? lme_internal_launch_sdp_rows(arg, re, &a, h->srows_lds, st)
                       : lme_internal_launch_sdp(which, arg, &a, st);
    return e == hipSuccess ? LME_OK : hip_fail(e, "launch streamed DOPRI5");
  };
  hipError_t e = hipMemcpyAsync(a.rho, rho0_dev, (size_t)h->state_elems * 16,
                                hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "copy rho0");
  if ((rc = L(4, 0, s)) || (rc = L(3, -1, s))) return rc;
  if (a.n_stops > 0) {
    if (opt->h0 <= 0.0) {
      if ((rc = L(5, 0, s)) || (rc = L(6, 0, s)) || (rc = L(7, 0, s)) || (rc = L(8, 0, s)) ||
          (rc = L(9, 0, s)))
        return rc;
    } else if ((rc = L(9, 1, s))) {
      return rc;
    }
    rc = cached_graph(h, &a, sizeof a, [&](hipStream_t gs) -> int {
      int r = 0;
      for (int st = 0; st < 7 && !r; ++st) r = L(0, st, gs);
      if (!r) r = L(1, 0, gs);
      if (!r) r = L(2, 0, gs);
      if (!r) r = L(3, -1, gs);
      return r;
    });
    if (rc) return rc;
    constexpr int kReplay = 16;
    for (int64_t done = 0; done <= opt->max_steps; done += kReplay) {
      for (int r = 0; r < kReplay; ++r)
        if ((e = hipGraphLaunch(h->gexec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
      if ((e = hipMemcpyAsync(h->h_active, a.n_active, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
          (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, "poll active count");
      if (*h->h_active == 0) break;
    }
  }
  if ((rc = L(10, 0, s))) return rc;
  if (rho_out_dev &&
      (e = hipMemcpyAsync(rho_out_dev, a.rho, (size_t)h->state_elems * 16,
                          hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "copy rho");
  return LME_OK;
}

// Streamed fixed-step RK4: a graph of kGraphSteps steps (4 stage kernels,
// outputs, counter update each) replayed ceil(nsteps / kGraphSteps) times;
// steps past nsteps do nothing.
static int evolve_rk4_streamed(lme_ctx *h, int32_t n_t, int32_t nsteps, double hstep,
                               const double *u_dev, const void *rho0_dev, void *expect_dev,
                               void *states_dev, void *rho_out_dev, int64_t *counts_dev,
                               int32_t *status_dev, hipStream_t s) {
  lme::StreamArgs a;
  std::memset(&a, 0, sizeof a);
  int rc = stream_workspace(h, &a);
  if (rc) return rc;
  a.u = u_dev ? u_dev : static_cast<const double *>(h->d_u.p);
  a.n_t = n_t;
  a.seg_of_step = static_cast<const int32_t *>(h->d_steps.p);
  a.out_step = a.seg_of_step + nsteps;
  a.nsteps = nsteps;
  a.h = hstep;
  a.states = static_cast<double *>(states_dev);
  a.expect = static_cast<double *>(expect_dev);
  a.counts = counts_dev;
  a.status = status_dev;
  auto L = [&](int which, int arg, hipStream_t st) -> int {
    hipError_t e = lme_internal_launch_sdp(which, arg, &a, st);
    return e == hipSuccess ? LME_OK : hip_fail(e, "launch streamed RK4");
  };
  hipError_t e = hipMemcpyAsync(a.rho, rho0_dev, (size_t)h->state_elems * 16,
                                hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "copy rho0");
  if ((rc = L(22, 1, s)) || (rc = L(3, 0, s))) return rc;   // counters, outputs at t0
  if (nsteps > 0) {
    constexpr int kGraphSteps = 16;
    const int per = std::min(nsteps, kGraphSteps);
    rc = cached_graph(h, &a, sizeof a, [&](hipStream_t gs) -> int {
      int r = 0;
      for (int q = 0; q < per && !r; ++q) {
        for (int st = 0; st < 4 && !r; ++st) r = L(20, st, gs);
        if (!r) r = L(21, 0, gs);
        if (!r) r = L(22, 0, gs);
      }
      return r;
    });
    if (rc) return rc;
    for (int done = 0; done < nsteps; done += per)
      if ((e = hipGraphLaunch(h->gexec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  if ((rc = L(22, 2, s))) return rc;
  if (rho_out_dev &&
      (e = hipMemcpyAsync(rho_out_dev, a.rho, (size_t)h->state_elems * 16,
                          hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "copy rho");
  return LME_OK;
}

static int evolve_dp5(lme_handle h, const lme_options *opt, int32_t n_t, const double *tlist,
                      const void *rho0_dev, const double *u_dev, void *expect_dev,
                      void *states_dev, void *rho_out_dev, int64_t *counts_dev,
                      int32_t *status_dev, void *stream, bool noalloc) {
  if (!(opt->rtol > 0.0) || !std::isfinite(opt->rtol) || !(opt->atol >= 0.0) ||
      !std::isfinite(opt->atol))
    return fail(LME_EINVAL, "DOPRI5 needs rtol > 0 and atol >= 0, finite");
  if (!std::isfinite(opt->h0) || !(opt->h_min >= 0.0) || !std::isfinite(opt->h_min))
    return fail(LME_EINVAL, "DOPRI5 needs a finite h0 and h_min >= 0");
  if (opt->max_steps < 1) return fail(LME_EINVAL, "DOPRI5 needs max_steps >= 1");
  if (opt->block != 0 && opt->block != 512 && opt->block != 1024)
    return fail(LME_EINVAL, "the adaptive stepper runs 512-thread workgroups (1024 in the "
                "column layout)");
  std::vector<double> stops;
  std::vector<int32_t> out_idx, seg;
  int rc = dp5_tables(h, n_t, tlist, &stops, &out_idx, &seg);
  if (rc) return rc;
  int max_n2 = 0;
  for (auto &d : h->inst) max_n2 = std::max(max_n2, d.n * d.n);
  int epts[16];
  const int ne = lme_internal_dp5_epts(epts, 16);
  int EPT = 0;
  for (int i = 0; i < ne && !EPT; ++i)
    if (512 * epts[i] >= max_n2) EPT = epts[i];
  if (!EPT && opt->path == LME_PATH_RESIDENT)
    return fail(LME_ENOTSUP, "largest instance (%d elements) exceeds the resident adaptive "
                "workgroup", max_n2);
  bool streamed = opt->path == LME_PATH_STREAMED || !EPT;
  // column-owner resident kernel: the column-kernel shapes, up to 16 rows per
  // thread
  // (1024 threads with 4 rows per thread, else 512 threads)
  int wo = 0, nc = 0, nb = 0, col_ept = 0;
  auto col_T = [](int e) { return e == 4 ? 1024 : 512; };
  if (opt->layout != LME_LAYOUT_ROW && opt->path != LME_PATH_STREAMED &&
      column_eligible(h, &wo, &nc, &nb))
    for (int e : {4, 8, 16})
      if (!col_ept && (opt->block == 0 || opt->block == col_T(e)) &&
          column_fits(h, col_T(e), e, false))
        col_ept = e;
  if (opt->layout == LME_LAYOUT_COLUMN && !col_ept)
    return fail(LME_ENOTSUP, "the batch has no column-owner adaptive kernel (operator shape, "
                "dimension or path)");
  // AUTO: the column kernel with 4 (1024 threads) or 8 rows per thread; the
  // 16-row variant keeps fewer operands in registers and is not faster than
  // the row kernel
  if (opt->layout == LME_LAYOUT_AUTO && col_ept == 16) col_ept = 0;
  if (noalloc && streamed && !col_ept)
    return fail(LME_ENOTSUP, "lme_evolve_noalloc runs the resident kernels only; this batch "
                "needs the streamed adaptive path");

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (noalloc && !h->on_device)
    return fail(LME_EINVAL, "the handle was created without a device: its operators are not on "
                "a GPU");
  if ((rc = ensure_device(h))) return rc;
  // tables: [stops | out_idx | seg], content-cached
  const size_t ns = stops.size();
  std::vector<uint8_t> buf(ns * 8 + 2 * ns * 4 + 16, 0);
  if (ns) {
    std::memcpy(buf.data(), stops.data(), ns * 8);
    std::memcpy(buf.data() + ns * 8, out_idx.data(), ns * 4);
    std::memcpy(buf.data() + ns * 12, seg.data(), ns * 4);
  }
  if (!noalloc) {
    std::vector<double> key(stops);
    key.push_back((double)n_t);
    for (int k = 0; k < n_t; ++k) key.push_back(tlist[k]);
    if (key != h->stops_key || !h->d_stops.p) {
      if ((rc = h->d_stops.upload(buf.data(), buf.size(), "stop tables"))) return rc;
      h->stops_key.swap(key);
    }
  }
  Plan *plan = nullptr;
  if (col_ept) {
    streamed = false;
    if ((rc = plan_packs(h, col_T(col_ept), col_ept, 0, col_T(col_ept) * col_ept, 1, 1, &plan, 0,
                         !noalloc)))
      return rc;
  } else if (!streamed) {
    rc = plan_packs(h, 512, EPT, 0, 512 * EPT, 0, 1, &plan, 0, !noalloc);
    if (rc == LME_ENOTSUP && opt->path == LME_PATH_AUTO && !noalloc)
      streamed = true;  // a pack does not fit in LDS
    else if (rc)
      return rc;
  }
  NoAlloc na;
  const uint8_t *tb = static_cast<const uint8_t *>(h->d_stops.p);
  double *kbuf = static_cast<double *>(h->d_kbuf.p);
  if (noalloc) {
    if ((rc = noalloc_stage(h, buf.data(), buf.size(), plan, (size_t)7 * h->state_elems * 16, s,
                            &na)))
      return rc;
    tb = na.base;
    kbuf = reinterpret_cast<double *>(na.base + na.kbuf_off);
  }

  if (!streamed && !noalloc) {
    const size_t kbytes = (size_t)7 * h->state_elems * 16;
    if (h->d_kbuf.bytes < kbytes) {
      h->d_kbuf.release();
      hipError_t e = hipMalloc(&h->d_kbuf.p, kbytes);
      if (e != hipSuccess) {
        h->d_kbuf.p = nullptr;
        return fail(LME_ENOMEM, "hipMalloc(stage derivatives, %zu B) failed", kbytes);
      }
      h->d_kbuf.bytes = kbytes;
    }
    kbuf = static_cast<double *>(h->d_kbuf.p);
  }

  lme::Dp5Args a;
  std::memset(&a, 0, sizeof a);
  a.packs = plan ? static_cast<const PackDesc *>(plan->d_packs.p) : nullptr;
  a.order = plan ? static_cast<const int32_t *>(plan->d_order.p) : nullptr;
  if (noalloc) {
    a.packs = reinterpret_cast<const PackDesc *>(na.base + na.packs_off);
    a.order = reinterpret_cast<const int32_t *>(na.base + na.order_off);
  }
  a.inst = static_cast<const InstDesc *>(h->d_inst.p);
  a.ops = static_cast<const uint8_t *>(h->d_ops.p);
  a.eops = static_cast<const uint8_t *>(h->d_eops.p);
  a.u = u_dev ? u_dev : static_cast<const double *>(h->d_u.p);
  a.n_ctrl = h->n_ctrl;
  a.n_seg = h->n_seg;
  a.n_e = h->n_e;
  a.n_t = n_t;
  a.stops = reinterpret_cast<const double *>(tb);
  a.stop_out = reinterpret_cast<const int32_t *>(tb + ns * 8);
  a.stop_seg = reinterpret_cast<const int32_t *>(tb + ns * 12);
  a.n_stops = (int32_t)ns;
  a.t0 = tlist[0];
  a.rtol = opt->rtol;
  a.atol = opt->atol;
  a.h0 = opt->h0;
  a.h_min = opt->h_min;
  a.max_steps = opt->max_steps;
  a.state_elems = h->state_elems;
  a.kbuf = kbuf;
  a.rho0 = static_cast<const double *>(rho0_dev);
  a.rho_out = static_cast<double *>(rho_out_dev);
  a.states = static_cast<double *>(states_dev);
  a.expect = static_cast<double *>(expect_dev);
  a.counts = counts_dev;
  a.status = status_dev;
  if (streamed)
    return evolve_dp5_streamed(h, opt, n_t, tlist, rho0_dev, u_dev, expect_dev, states_dev,
                               rho_out_dev, counts_dev, status_dev, s, a);
  hipError_t e = col_ept ? lme_internal_launch_dp5_col(col_ept, wo, nc, nb, real_structure(h), &a,
                                                       (int)plan->packs.size(), plan->max_lds, s)
                         : lme_internal_launch_dp5(EPT, &a, (int)plan->packs.size(),
                                                   plan->max_lds, s);
  if (e != hipSuccess) return hip_fail(e, "launch resident DOPRI5");
  return LME_OK;
}

static int evolve_impl(lme_handle h, const lme_options *opt, int32_t n_t, const double *tlist,
                       const void *rho0_dev, const double *u_dev, void *expect_dev,
                       void *states_dev, void *rho_out_dev, int64_t *counts_dev,
                       int32_t *status_dev, void *stream, bool noalloc) {
  if (!h) return fail(LME_EINVAL, "handle is NULL");
  if (!opt) return fail(LME_EINVAL, "options are NULL");
  if (!rho0_dev) return fail(LME_EINVAL, "rho0 is NULL");
  int rc = check_times(n_t, tlist);
  if (rc) return rc;
  if (opt->path < LME_PATH_AUTO || opt->path > LME_PATH_STREAMED)
    return fail(LME_EINVAL, "unknown path %d", opt->path);
  if (opt->block != 0 && opt->block != 256 && opt->block != 512 && opt->block != 768 &&
      opt->block != 1024)
    return fail(LME_EINVAL, "block must be 0, 256, 512, 768 or 1024");
  if (opt->hermitian != 0 && opt->hermitian != 1)
    return fail(LME_EINVAL, "hermitian must be 0 or 1");
  if (opt->layout < LME_LAYOUT_AUTO || opt->layout > LME_LAYOUT_COLUMN)
    return fail(LME_EINVAL, "unknown layout %d", opt->layout);
  if (!h->fn.empty()) {
    if (opt->method == LME_DOPRI5)
      return fail(LME_ENOTSUP, "closed-form amplitudes are integrated with fixed-step RK4 only");
    if (opt->path == LME_PATH_STREAMED)
      return fail(LME_ENOTSUP, "closed-form amplitudes run on the resident kernels only");
    if (u_dev)
      return fail(LME_EINVAL, "u_dev overrides piecewise amplitudes; this handle has "
                  "closed-form amplitudes");
  }
  if (opt->method == LME_DOPRI5)
    return evolve_dp5(h, opt, n_t, tlist, rho0_dev, u_dev, expect_dev, states_dev, rho_out_dev,
                      counts_dev, status_dev, stream, noalloc);
  if (opt->method != LME_RK4) return fail(LME_EINVAL, "unknown method %d", opt->method);
  if (n_t > 1 && opt->nsteps < 1) return fail(LME_EINVAL, "RK4 needs nsteps >= 1");
  const int32_t nsteps = n_t > 1 ? opt->nsteps : 0;
  const double hstep = n_t > 1 ? (tlist[n_t - 1] - tlist[0]) / nsteps : 0.0;
  std::vector<int32_t> tab;
  if ((rc = rk4_tables(h, n_t, tlist, nsteps, hstep, &tab))) return rc;
  lme_options tuned = *opt;  // tuned defaults fill the fields left open
  const bool herm = opt->hermitian == 1;
  const int tl_layout = herm ? h->tuning.herm_layout : h->tuning.rk4_layout;
  const int tl_block = herm ? h->tuning.herm_block : h->tuning.rk4_block;
  if (tuned.layout == LME_LAYOUT_AUTO && tuned.block == 0 && tl_block > 0) {
    tuned.layout = tl_layout;
    tuned.block = tl_block;
  }
  opt = &tuned;
  // column layout: T in {512, 768} (also Hermitian); row layout:
  // T in {256, 512, 1024}
  int T = 0, EPT = 0, column = 0, col_cfg = -1, wo = 0, nc = 0, nb = 0, pack_cap = 0;
  const int re = real_structure(h);
  // With control terms the full-path column kernels run short of registers:
  // AUTO takes the row layout there (1.3 - 1.8x faster on driven JC batches
  // of 256 to 4096 instances, n = 12 to 40; equal at 64 instances, n = 60).
  if (opt->layout != LME_LAYOUT_ROW && column_eligible(h, &wo, &nc, &nb) &&
      (nb == 0 || herm || opt->layout == LME_LAYOUT_COLUMN)) {
    for (int c = 1; c >= 0; --c) {   // prefer the larger workgroup
      const int cT = herm ? lme::kHermCfg[c][0] : lme::kColCfg[c][0];
      const int cE = herm ? lme::kHermCfg[c][1] : lme::kColCfg[c][1];
      if ((opt->block == 0 || opt->block == cT) && column_fits(h, cT, cE, herm)) {
        T = cT;
        EPT = cE;
        column = herm ? 2 : 1;
        col_cfg = c;
        break;
      }
    }
  }
  bool streamed = opt->path == LME_PATH_STREAMED;
  if (!column && !streamed) {
    if (opt->layout == LME_LAYOUT_COLUMN)
      return fail(LME_ENOTSUP, "the column layout does not cover these operators / block size");
    if (opt->block == 768) return fail(LME_EINVAL, "block 768 exists only in the column layout");
    // the row layout has no Hermitian variant: it computes every element
    rc = pick_rk4_config(h, opt->block, &T, &EPT, &pack_cap);
    if (rc == LME_ENOTSUP && opt->path == LME_PATH_AUTO && !noalloc && h->fn.empty())
      streamed = true;  // an instance is too large for a resident workgroup
    else if (rc)
      return rc;
  }
  if (noalloc && streamed)
    return fail(LME_ENOTSUP, "lme_evolve_noalloc runs the resident kernels only");
  if (noalloc && !h->on_device)
    return fail(LME_EINVAL, "the handle was created without a device: its operators are not on "
                "a GPU");

  // validation done: from here on the device is used
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = ensure_device(h))) return rc;
  if (!noalloc && (rc = upload_tables(h, tab, s))) return rc;
  hipError_t e;
  Plan *plan = nullptr;
  if (!streamed) {
    rc = plan_packs(h, T, EPT, 0, pack_cap > 0 ? pack_cap : T * EPT, column, 0, &plan, 0,
                    !noalloc);
    if (rc == LME_ENOTSUP && opt->path == LME_PATH_AUTO && !column && !noalloc && h->fn.empty())
      streamed = true;
    else if (rc)
      return rc;
  }
  if (streamed)
    return evolve_rk4_streamed(h, n_t, nsteps, hstep, u_dev, rho0_dev, expect_dev, states_dev,
                               rho_out_dev, counts_dev, status_dev, s);
  NoAlloc na;
  if (noalloc &&
      (rc = noalloc_stage(h, tab.data(), tab.size() * sizeof(int32_t), plan, 0, s, &na)))
    return rc;

  lme::Rk4Args a;
  std::memset(&a, 0, sizeof a);
  a.packs = static_cast<const PackDesc *>(plan->d_packs.p);
  a.order = static_cast<const int32_t *>(plan->d_order.p);
  a.inst = static_cast<const InstDesc *>(h->d_inst.p);
  a.ops = static_cast<const uint8_t *>(h->d_ops.p);
  a.adjoint = 0;
  a.eops = static_cast<const uint8_t *>(h->d_eops.p);
  a.u = u_dev ? u_dev : static_cast<const double *>(h->d_u.p);
  a.n_ctrl = h->n_ctrl;
  a.n_seg = h->n_seg;
  a.n_e = h->n_e;
  a.n_t = n_t;
  a.seg_of_step = static_cast<const int32_t *>(h->d_steps.p);
  a.out_step = static_cast<const int32_t *>(h->d_steps.p) + nsteps;
  if (noalloc) {
    a.packs = reinterpret_cast<const PackDesc *>(na.base + na.packs_off);
    a.order = reinterpret_cast<const int32_t *>(na.base + na.order_off);
    a.seg_of_step = reinterpret_cast<const int32_t *>(na.base);
    a.out_step = reinterpret_cast<const int32_t *>(na.base) + nsteps;
  }
  a.nsteps = nsteps;
  a.h = hstep;
  a.fn = h->fn.empty() ? nullptr : static_cast<const double *>(h->d_fn.p);
  a.t0 = tlist[0];
  a.state_elems = h->state_elems;
  a.rho0 = static_cast<const double *>(rho0_dev);
  a.rho_out = static_cast<double *>(rho_out_dev);
  a.states = static_cast<double *>(states_dev);
  a.expect = static_cast<double *>(expect_dev);
  a.counts = counts_dev;
  a.status = status_dev;
  // one-wavefront packs of small instances: one element per lane, the stage
  // input exchanged between lanes
  bool lane = !column && T == 64 && EPT == 1;
  for (auto &d : h->inst)
    lane = lane && lme_internal_lane_fits(d.fwd.wo, d.fwd.nb, d.fwd.wb, d.fwd.nc, d.fwd.wc);
  if (column)
    e = lme_internal_launch_rk4_colown(col_cfg, column == 2, wo, nc, nb, re, &a,
                                       (int)plan->packs.size(), plan->max_lds, s);
  else if (lane)
    e = lme_internal_launch_rk4_lane(&a, (int)plan->packs.size(), plan->max_lds, s);
  else
    e = lme_internal_launch_rk4(T, EPT, &a, (int)plan->packs.size(), plan->max_lds, s);
  if (e != hipSuccess) return hip_fail(e, "launch resident RK4");
  return LME_OK;
}

extern "C" int lme_evolve(lme_handle h, const lme_options *opt, int32_t n_t, const double *tlist,
                          const void *rho0_dev, const double *u_dev, void *expect_dev,
                          void *states_dev, void *rho_out_dev, int64_t *counts_dev,
                          int32_t *status_dev, void *stream) {
  try {
    return evolve_impl(h, opt, n_t, tlist, rho0_dev, u_dev, expect_dev, states_dev, rho_out_dev,
                       counts_dev, status_dev, stream, false);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

extern "C" int lme_evolve_noalloc(lme_handle h, const lme_options *opt, int32_t n_t,
                                  const double *tlist, const void *rho0_dev, const double *u_dev,
                                  void *expect_dev, void *states_dev, void *rho_out_dev,
                                  int64_t *counts_dev, int32_t *status_dev, void *stream) {
  try {
    return evolve_impl(h, opt, n_t, tlist, rho0_dev, u_dev, expect_dev, states_dev, rho_out_dev,
                       counts_dev, status_dev, stream, true);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

// ---------------------------------------------------------------------------
// single application
// ---------------------------------------------------------------------------
static bool column_eligible(const lme_ctx *h, int *wo, int *nc, int *nb);
static int real_structure(const lme_ctx *h);

// Element tiles of the streamed kernels: 2048 consecutive elements of one
// instance each, in instance order.
constexpr int kTileElems = 2048;

static int ensure_tiles(lme_ctx *h) {
  if (h->d_tiles.p) return LME_OK;
  // every instance 128 <= n <= 256: tiles of 16 whole rows, for the
  // row-block stage kernel of the adaptive stepper; else kTileElems elements
  int max_n = 0, min_n = 1 << 30, wo = 0, ncw = 0;
  for (auto &d : h->inst) {
    max_n = std::max(max_n, d.n);
    min_n = std::min(min_n, d.n);
    wo = std::max(wo, (int)d.fwd.wo);
    ncw = std::max(ncw, (int)(d.fwd.nc * d.fwd.wc));
  }
  const int64_t rows_lds = 16LL * 16 * max_n + 16LL * 16 * (1 + wo + ncw) + 4LL * 16 * (wo + ncw);
  h->srows_lds = (min_n >= 128 && max_n <= 256 && rows_lds <= h->lds_limit) ? (int)rows_lds : 0;
  std::vector<lme::Tile> t;
  for (int b = 0; b < h->n_inst; ++b) {
    const int n = h->inst[b].n, n2 = n * n;
    const int step = h->srows_lds ? 16 * n : kTileElems;
    for (int e0 = 0; e0 < n2; e0 += step) {
      lme::Tile x;
      x.inst = b;
      x.e0 = e0;
      x.e1 = std::min(n2, e0 + step);
      x.pad = 0;
      t.push_back(x);
    }
  }
  int rc = h->d_tiles.upload(t.data(), t.size() * sizeof(lme::Tile), "tiles");
  if (rc) return rc;
  h->tiles.swap(t);
  return LME_OK;
}

// Tiles of the streamed application: fixed kTileElems-element chunks of the
// packed state buffer (spanning instances), each with its first instance.
static int ensure_packed_tiles(lme_ctx *h) {
  if (h->d_ptiles.p) return LME_OK;
  std::vector<lme::Tile> t;
  int b = 0;
  for (int64_t e0 = 0; e0 < h->state_elems; e0 += kTileElems) {
    while (h->offsets[b] + (int64_t)h->dims[b] * h->dims[b] <= e0) ++b;
    lme::Tile x;
    x.inst = b;
    x.e0 = (int32_t)e0;
    x.e1 = (int32_t)std::min<int64_t>(h->state_elems, e0 + kTileElems);
    x.pad = 0;
    t.push_back(x);
  }
  int rc = h->d_ptiles.upload(t.data(), t.size() * sizeof(lme::Tile), "packed tiles");
  if (rc) return rc;
  h->n_ptiles = (int32_t)t.size();
  return LME_OK;
}

// Row blocks for the row-block application: 16 rows when every instance has
// n <= 256, else 4 (n <= 1024), so a block stages at most 64 KB.  Instances
// below n = 128 are left to the pack kernels, which serve them better.
static int ensure_row_tiles(lme_ctx *h) {
  if (h->rtile_R) return LME_OK;
  int max_n = 0, min_n = 1 << 30;
  for (int32_t n : h->dims) {
    max_n = std::max(max_n, n);
    min_n = std::min(min_n, n);
  }
  if (min_n < 128 || max_n > 1024) {
    h->rtile_R = -1;
    return LME_OK;
  }
  const int R = max_n <= 256 ? 16 : 4;
  std::vector<lme::Tile> t;
  for (int b = 0; b < h->n_inst; ++b)
    for (int r0 = 0; r0 < h->dims[b]; r0 += R) {
      lme::Tile x;
      x.inst = b;
      x.e0 = r0;
      x.e1 = std::min(r0 + R, h->dims[b]);
      x.pad = 0;
      t.push_back(x);
    }
  int rc = h->d_rtiles.upload(t.data(), t.size() * sizeof(lme::Tile), "row tiles");
  if (rc) return rc;
  // LDS: R rows of y and the row-side entries of the block's rows (complex
  // D, Oval, Jval; int Ocol, Jcol) for the widest forward or adjoint operator
  int wo = 0, ncw = 0;
  for (auto &d : h->inst)
    for (const lme::Signature *sg : {&d.fwd, &d.adj}) {
      wo = std::max(wo, (int)sg->wo);
      ncw = std::max(ncw, (int)(sg->nc * sg->wc));
    }
  const int64_t lds = 16LL * R * max_n + 16LL * R * (1 + wo + ncw) + 4LL * R * (wo + ncw);
  if (lds > h->lds_limit) {
    h->rtile_R = -1;
    return LME_OK;
  }
  h->n_rtiles = (int32_t)t.size();
  h->rtile_R = R;
  h->rtile_lds = (int32_t)lds;
  return LME_OK;
}

// Streamed application (stage input and result in HBM).  rows: allow the
// row-block kernel (every instance 128 <= n <= 1024); otherwise, and for the
// explicit streamed form, every element gathers straight from memory.
// Controls of an application at time t: the caller's or the create-time
// piecewise amplitudes with the segment holding t, or, with closed-form
// amplitudes, u(t) evaluated here into a one-segment table.
struct ApplyCtl {
  const double *u;
  int n_seg, seg;
};

static int apply_controls(lme_ctx *h, double t, const double *u_dev, hipStream_t s,
                          ApplyCtl *c) {
  if (h->fn.empty()) {
    c->u = u_dev ? u_dev : static_cast<const double *>(h->d_u.p);
    c->n_seg = h->n_seg;
    c->seg = segment_at(h, t);
    return LME_OK;
  }
  std::vector<double> uval((size_t)h->n_inst * h->n_ctrl);
  for (size_t q = 0; q < uval.size(); ++q) uval[q] = lme::coeff_fn_at(h->fn.data() + 7 * q, t);
  if (uval != h->fnu_key || !h->d_fnu.p) {
    int rc = h->d_fnu.upload(uval.data(), uval.size() * sizeof(double), "amplitudes at t");
    if (rc) return rc;
    h->fnu_key.swap(uval);
  }
  (void)s;
  c->u = static_cast<const double *>(h->d_fnu.p);
  c->n_seg = 1;
  c->seg = 0;
  return LME_OK;
}

static int apply_streamed(lme_ctx *h, int adjoint, double t, const double *u_dev,
                          const void *y_dev, void *out_dev, hipStream_t s, bool rows) {
  if (h->state_elems >= (int64_t)1 << 31)
    return fail(LME_ENOTSUP, "the streamed application addresses states below 2^31 elements");
  int rc = rows ? ensure_row_tiles(h) : LME_OK;
  if (rc) return rc;
  rows = rows && h->rtile_R > 0;
  if (!rows && (rc = ensure_packed_tiles(h))) return rc;
  lme::ApplyGArgs a;
  std::memset(&a, 0, sizeof a);
  a.tiles = static_cast<const lme::Tile *>(h->d_ptiles.p);
  a.n_tiles = h->n_ptiles;
  a.inst = static_cast<const InstDesc *>(h->d_inst.p);
  a.adjoint = adjoint;
  a.ops = static_cast<const uint8_t *>(adjoint ? h->d_adj.p : h->d_ops.p);
  ApplyCtl ctl;
  if ((rc = apply_controls(h, t, u_dev, s, &ctl))) return rc;
  a.u = ctl.u;
  a.n_ctrl = h->n_ctrl;
  a.n_seg = ctl.n_seg;
  a.seg = ctl.seg;
  a.y = static_cast<const double *>(y_dev);
  a.out = static_cast<double *>(out_dev);
  if (rows) {
    a.tiles = static_cast<const lme::Tile *>(h->d_rtiles.p);
    a.n_tiles = h->n_rtiles;
    hipError_t e = lme_internal_launch_apply_rows(h->rtile_R, adjoint ? 0 : real_structure(h), &a,
                                                  h->rtile_lds, s);
    return e == hipSuccess ? LME_OK : hip_fail(e, "launch row-block apply");
  }
  hipError_t e = lme_internal_launch_apply_global(&a, s);
  return e == hipSuccess ? LME_OK : hip_fail(e, "launch streamed apply");
}

// Superoperator of one instance in row-major vectorisation, vec(y)[i*n+j] =
// y_ij:  S = A (x) I + I (x) conj(A) + sum_k C_k (x) conj(C_k), i.e. row (i, j)
// holds A_il at column (l, j), conj(A_jl) at (i, l) and C_il conj(C_jm) at
// (l, m) -- the operator form L y = A y + y A^+ + sum_k C_k y C_k^+ written
// out element by element.
static void superop_rows(const Sparse &A, const std::vector<Sparse> &C,
                         std::vector<std::vector<std::pair<int, cd>>> *rows) {
  const int n = A.n;
  rows->assign((size_t)n * n, {});
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      std::vector<std::pair<int, cd>> r;
      for (auto &x : A.rows[i]) r.emplace_back(x.first * n + j, x.second);
      for (auto &x : A.rows[j]) r.emplace_back(i * n + x.first, std::conj(x.second));
      for (auto &c : C)
        for (auto &x : c.rows[i])
          for (auto &z : c.rows[j]) r.emplace_back(x.first * n + z.first, x.second * std::conj(z.second));
      std::sort(r.begin(), r.end(), [](const std::pair<int, cd> &a, const std::pair<int, cd> &b) {
        return a.first < b.first;
      });
      std::vector<std::pair<int, cd>> m;
      for (auto &e : r) {
        if (!m.empty() && m.back().first == e.first)
          m.back().second += e.second;
        else
          m.push_back(e);
      }
      (*rows)[(size_t)i * n + j].swap(m);
    }
}

static int ensure_superop(lme_ctx *h) {
  if (h->d_sd.p) return LME_OK;
  std::vector<lme::SuperDesc> sd(h->n_inst);
  std::vector<int32_t> col;
  std::vector<cd> val;
  for (int b = 0; b < h->n_inst; ++b) {
    std::vector<std::vector<std::pair<int, cd>>> rows;
    superop_rows(h->A_host[b], h->C_host[b], &rows);
    int w = 0;
    for (auto &r : rows) w = std::max(w, (int)r.size());
    const size_t n2 = rows.size();
    sd[b].col_off = (int64_t)col.size();
    sd[b].val_off = (int64_t)val.size();
    sd[b].w = w;
    sd[b].pad = 0;
    const size_t base_c = col.size(), base_v = val.size();
    col.resize(base_c + (size_t)w * n2);
    val.resize(base_v + (size_t)w * n2, cd(0.0, 0.0));
    for (size_t e = 0; e < n2; ++e)
      for (int sl = 0; sl < w; ++sl) {
        const bool on = sl < (int)rows[e].size();
        col[base_c + (size_t)sl * n2 + e] = on ? rows[e][sl].first : (int32_t)e;
        if (on) val[base_v + (size_t)sl * n2 + e] = rows[e][sl].second;
      }
  }
  int rc;
  if ((rc = h->d_sd.upload(sd.data(), sd.size() * sizeof(lme::SuperDesc), "superop index"))) return rc;
  if ((rc = h->d_scol.upload(col.data(), col.size() * 4, "superop columns"))) return rc;
  if ((rc = h->d_sval.upload(val.data(), val.size() * 16, "superop values"))) return rc;
  return LME_OK;
}

// Pipelined column application: row records of every instance (the layout
// of the device's Rec<wo, nc, nb>) in HBM, and the tile list.  Instances
// whose y and records fit a stage go whole, several of one signature per
// tile; larger ones are cut into row tiles, each staged with the band of
// rows its products read.  LME_ENOTSUP when an operator is too wide for a
// row tile to fit a stage.
static int ensure_pipe(lme_ctx *h, int wo, int nc, int nb) {
  if (h->pipe_state == 1) return LME_OK;
  if (h->pipe_state == -1) return LME_ENOTSUP;
  h->pipe_state = -1;
  const int S = lme::rec_bytes(wo, nc, nb), H = lme::rec_hdr_bytes(wo, nc, nb);
  const int NH = 1 + wo + nc + nb * lme::kColWB;
  const int CB = 1 + wo + nc, CQ = 1 + lme::kColWB;
  // records
  std::vector<int64_t> roff(h->n_inst);
  int64_t total = 0;
  for (int b = 0; b < h->n_inst; ++b) {
    roff[b] = total;
    total += (int64_t)h->inst[b].n * S;
  }
  std::vector<uint8_t> recs((size_t)total, 0);
  std::vector<std::vector<int32_t>> lo(h->n_inst), hi(h->n_inst);
  for (int b = 0; b < h->n_inst; ++b) {
    const InstDesc &d = h->inst[b];
    const lme::Signature &g = d.fwd;
    const int n = g.n, n16 = 16 * n;
    const lme::BlobLayout L = lme::blob_layout(n, g.wo, g.nb, g.wb, g.nc, g.wc);
    const uint8_t *blob = h->ops.data() + d.ops_off;
    auto val = [&](int off, int idx) {
      double v[2];
      std::memcpy(v, blob + off + 16 * idx, 16);
      return std::pair<double, double>(v[0], v[1]);
    };
    auto col = [&](int off, int idx) {
      int32_t c;
      std::memcpy(&c, blob + off + 4 * idx, 4);
      return c;
    };
    lo[b].resize(n);
    hi[b].resize(n);
    for (int i = 0; i < n; ++i) {
      uint8_t *r = recs.data() + roff[b] + (size_t)i * S;
      int32_t hd[32] = {0};
      std::vector<std::pair<double, double>> v((size_t)(S - H) / 16, {0.0, 0.0});
      int l = i, u = i;
      auto ref = [&](int c) { l = std::min(l, c); u = std::max(u, c); return c * n16; };
      hd[0] = i * n16;
      v[0] = val(L.offD, i);
      for (int w = 0; w < wo; ++w) {
        hd[1 + w] = ref(col(L.offOcol, w * n + i));
        v[1 + w] = val(L.offOval, w * n + i);
      }
      for (int k = 0; k < nc; ++k) {
        hd[1 + wo + k] = ref(col(L.offJcol, k * n + i));
        v[1 + wo + k] = val(L.offJval, k * n + i);
      }
      for (int q = 0; q < nb; ++q) {
        v[CB + q * CQ] = val(L.offDB, q * n + i);
        for (int w = 0; w < lme::kColWB; ++w) {
          const bool on = w < g.wb;
          hd[1 + wo + nc + q * lme::kColWB + w] =
              ref(on ? col(L.offOBcol, (q * g.wb + w) * n + i) : i);
          if (on) v[CB + q * CQ + 1 + w] = val(L.offOBval, (q * g.wb + w) * n + i);
        }
      }
      std::memcpy(r, hd, 4 * NH);
      for (size_t k = 0; k < v.size(); ++k) {
        std::memcpy(r + H + 16 * k, &v[k].first, 8);
        std::memcpy(r + H + 16 * k + 8, &v[k].second, 8);
      }
      lo[b][i] = l;
      hi[b][i] = u;
    }
  }
  // tiles
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<int32_t>> groups;
  for (int b = 0; b < h->n_inst; ++b) {
    const lme::Signature &g = h->inst[b].fwd;
    groups[std::make_tuple(g.n, g.wo, g.wb, g.nc, g.wc, g.nb)].push_back(b);
  }
  std::vector<lme::PTile> tiles;
  const int T = lme::kPipeT, stage = lme::kPipeStage;
  auto add = [&](lme::PTile &t, int k, int b) {
    t.yoff[k] = h->inst[b].rho_off;
    t.roff[k] = roff[b];
    t.id[k] = b;
  };
  for (auto &gr : groups) {
    const std::vector<int32_t> &ids = gr.second;
    const int n = std::get<0>(gr.first), wb = std::get<2>(gr.first);
    const int yb = 16 * n * n, rb = n * S;
    if (yb + rb <= stage && n <= T) {
      // at most kPipeEPT rows per thread: m n ceil(n / kPipeEPT) <= T
      const int m_max = std::min({stage / (yb + rb), T / (n * ((n + lme::kPipeEPT - 1) /
                                                                lme::kPipeEPT)),
                                  (int)ids.size(), lme::kPipeMaxM});
      const int cnt = (int)ids.size(), n_t = (cnt + m_max - 1) / m_max;
      int done = 0;
      for (int q = 0; q < n_t; ++q) {
        const int m = (cnt - done + (n_t - q) - 1) / (n_t - q);
        lme::PTile t;
        std::memset(&t, 0, sizeof t);
        t.m = m;
        t.n = n;
        t.G = std::min(T / (m * n), n);
        t.r0 = 0;
        t.r1 = n;
        t.h0 = 0;
        t.span = n;
        t.wb = wb;
        t.rec_lds = m * yb;
        for (int k = 0; k < m; ++k) add(t, k, ids[done + k]);
        tiles.push_back(t);
        done += m;
      }
    } else {
      const int max_span = (stage - rb) / (16 * n);
      const int max_rows = lme::kPipeEPT * (T / n);  // at most kPipeEPT rows per thread
      if (rb > stage / 2 || max_span < 1 || n > T) return LME_ENOTSUP;
      for (int b : ids) {
        int r0 = 0;
        while (r0 < n) {
          int l = lo[b][r0], u = hi[b][r0];
          if (u - l + 1 > max_span) return LME_ENOTSUP;  // one row's band is too wide
          int r1 = r0 + 1;
          while (r1 < n && r1 - r0 < max_rows) {
            const int l2 = std::min(l, lo[b][r1]), u2 = std::max(u, hi[b][r1]);
            if (u2 - l2 + 1 > max_span) break;
            l = l2;
            u = u2;
            ++r1;
          }
          lme::PTile t;
          std::memset(&t, 0, sizeof t);
          t.m = 1;
          t.n = n;
          t.G = std::min(T / n, r1 - r0);
          t.r0 = r0;
          t.r1 = r1;
          t.h0 = l;
          t.span = u - l + 1;
          t.wb = wb;
          t.rec_lds = t.span * 16 * n;
          add(t, 0, b);
          tiles.push_back(t);
          r0 = r1;
        }
      }
    }
  }
  // largest tiles first, so that the workgroups' round-robin shares even out
  std::vector<int> ord(tiles.size());
  for (size_t k = 0; k < ord.size(); ++k) ord[k] = (int)k;
  auto cost = [&](const lme::PTile &t) { return (int64_t)t.m * t.span * t.n; };
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int x, int y) { return cost(tiles[x]) > cost(tiles[y]); });
  std::vector<lme::PTile> sorted;
  for (int k : ord) sorted.push_back(tiles[k]);
  int rc;
  if ((rc = h->d_recs.upload(recs.data(), recs.size(), "row records"))) return rc;
  if ((rc = h->d_pt.upload(sorted.data(), sorted.size() * sizeof(lme::PTile), "tiles"))) return rc;
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute(CUs)");
  h->n_pipe = (int32_t)sorted.size();
  // one workgroup per CU; more when a workgroup would hold more descriptors
  // than its LDS table
  h->pipe_grid = std::min(h->n_pipe, std::max(cus, (h->n_pipe + lme::kPipeMaxTiles - 1) /
                                                       lme::kPipeMaxTiles));
  h->pipe_state = 1;
  return LME_OK;
}

static int apply_impl(lme_handle h, int32_t form, int32_t adjoint, double t, const double *u_dev,
                      const void *y_dev, void *out_dev, void *stream) {
  if (!h) return fail(LME_EINVAL, "handle is NULL");
  if (!y_dev || !out_dev) return fail(LME_EINVAL, "y and out must be device pointers");
  if (y_dev == out_dev) return fail(LME_EINVAL, "y and out must not overlap");
  if (!std::isfinite(t)) return fail(LME_EINVAL, "t is not finite");
  if (form != LME_FORM_OPERATOR && form != LME_FORM_SUPEROP && form != LME_FORM_OPERATOR_STREAMED)
    return fail(LME_EINVAL, "unknown form %d", form);
  if (form == LME_FORM_SUPEROP && (adjoint || h->n_ctrl > 0))
    return fail(LME_ENOTSUP, "the superoperator form is forward-only and takes no controls");
  if (u_dev && !h->fn.empty())
    return fail(LME_EINVAL, "u_dev overrides piecewise amplitudes; this handle has closed-form "
                "amplitudes");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc = ensure_device(h);
  if (rc) return rc;
  adjoint = adjoint ? 1 : 0;
  ApplyCtl ctl;
  if ((rc = apply_controls(h, t, u_dev, s, &ctl))) return rc;
  if (form == LME_FORM_SUPEROP) {
    if ((rc = ensure_superop(h)) || (rc = ensure_tiles(h))) return rc;
    lme::SuperArgs a;
    std::memset(&a, 0, sizeof a);
    a.tiles = static_cast<const lme::Tile *>(h->d_tiles.p);
    a.n_tiles = (int32_t)h->tiles.size();
    a.inst = static_cast<const InstDesc *>(h->d_inst.p);
    a.sd = static_cast<const lme::SuperDesc *>(h->d_sd.p);
    a.col = static_cast<const int32_t *>(h->d_scol.p);
    a.val = static_cast<const double *>(h->d_sval.p);
    a.y = static_cast<const double *>(y_dev);
    a.out = static_cast<double *>(out_dev);
    hipError_t e = lme_internal_launch_superop(&a, s);
    return e == hipSuccess ? LME_OK : hip_fail(e, "launch superoperator");
  }
  if (form == LME_FORM_OPERATOR_STREAMED)
    return apply_streamed(h, adjoint, t, u_dev, y_dev, out_dev, s, false);
  int wo, nc, nb;
  if (!adjoint && column_eligible(h, &wo, &nc, &nb) && h->apply_path == 0 &&
      2 * lme::kPipeStage + lme::kPipeMaxTiles * (int)sizeof(lme::PTile) + 16 <= h->lds_limit) {
    rc = ensure_pipe(h, wo, nc, nb);
    if (rc != LME_OK && rc != LME_ENOTSUP) return rc;
    if (rc == LME_OK) {
      lme::PipeArgs a;
      std::memset(&a, 0, sizeof a);
      a.tiles = static_cast<const lme::PTile *>(h->d_pt.p);
      a.n_tiles = h->n_pipe;
      a.recs = static_cast<const uint8_t *>(h->d_recs.p);
      a.u = ctl.u;
      a.n_ctrl = h->n_ctrl;
      a.n_seg = ctl.n_seg;
      a.seg = ctl.seg;
      a.y = static_cast<const double *>(y_dev);
      a.out = static_cast<double *>(out_dev);
      hipError_t e = lme_internal_launch_apply_pipe(wo, nc, nb, real_structure(h), &a,
                                                    h->pipe_grid, s);
      return e == hipSuccess ? LME_OK : hip_fail(e, "launch pipelined application");
    }
  }
  if (!adjoint && column_eligible(h, &wo, &nc, &nb)) {
    // column-owner application: apply_block threads, up to 64 rows per thread
    Plan *cp;
    const int T = h->apply_block;
    rc = plan_packs(h, T, 64, 0, T * 64, 3, 0, &cp, h->apply_lds_kb * 1024);
    if (rc == LME_OK) {
      lme::ApplyArgs a;
      std::memset(&a, 0, sizeof a);
      a.packs = static_cast<const PackDesc *>(cp->d_packs.p);
      a.order = static_cast<const int32_t *>(cp->d_order.p);
      a.inst = static_cast<const InstDesc *>(h->d_inst.p);
      a.ops = static_cast<const uint8_t *>(h->d_ops.p);
      a.u = ctl.u;
      a.n_ctrl = h->n_ctrl;
      a.n_seg = ctl.n_seg;
      a.seg = ctl.seg;
      a.y = static_cast<const double *>(y_dev);
      a.out = static_cast<double *>(out_dev);
      hipError_t e = lme_internal_launch_apply_col(T, wo, nc, nb, real_structure(h), &a,
                                                   (int)cp->packs.size(), cp->max_lds, s);
      return e == hipSuccess ? LME_OK : hip_fail(e, "launch column application");
    }
    if (rc != LME_ENOTSUP) return rc;
  }
  // packs of at most apply_cap elements: several workgroups per CU keep
  // enough HBM reads in flight
  Plan *plan;
  rc = plan_packs(h, 256, 0, adjoint, h->apply_cap, 0, 0, &plan);
  if (rc == LME_ENOTSUP) return apply_streamed(h, adjoint, t, u_dev, y_dev, out_dev, s, true);
  if (rc) return rc;
  lme::ApplyArgs a;
  std::memset(&a, 0, sizeof a);
  a.packs = static_cast<const PackDesc *>(plan->d_packs.p);
  a.order = static_cast<const int32_t *>(plan->d_order.p);
  a.inst = static_cast<const InstDesc *>(h->d_inst.p);
  a.adjoint = adjoint;
  a.ops = static_cast<const uint8_t *>(adjoint ? h->d_adj.p : h->d_ops.p);
  a.u = ctl.u;
  a.n_ctrl = h->n_ctrl;
  a.n_seg = ctl.n_seg;
  a.seg = ctl.seg;
  a.y = static_cast<const double *>(y_dev);
  a.out = static_cast<double *>(out_dev);
  hipError_t e;
  if (!adjoint && column_eligible(h, &wo, &nc, &nb))
    e = lme_internal_launch_apply_shape(wo, nc, nb, real_structure(h), &a,
                                        (int)plan->packs.size(), plan->max_lds, s);
  else
    e = lme_internal_launch_apply_lds(&a, (int)plan->packs.size(), plan->max_lds, s);
  if (e != hipSuccess) return hip_fail(e, "launch apply");
  return LME_OK;
}

extern "C" int lme_apply(lme_handle h, int32_t form, int32_t adjoint, double t,
                         const double *u_dev, const void *y_dev, void *out_dev, void *stream) {
  try {
    return apply_impl(h, form, adjoint, t, u_dev, y_dev, out_dev, stream);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

// ---------------------------------------------------------------------------
// cost and gradient (discrete adjoint of RK4)
// ---------------------------------------------------------------------------
static int cost_grad_impl(lme_handle h, int32_t nsteps, int32_t ckpt_every, double t0, double t1,
                          const void *rho0_dev, const void *O_dev, const double *u_dev,
                          double *cost_dev, double *grad_dev, void *stream) {
  if (!h) return fail(LME_EINVAL, "handle is NULL");
  if (!rho0_dev || !O_dev || !cost_dev || !grad_dev)
    return fail(LME_EINVAL, "rho0, O, cost and grad must be device pointers");
  if (nsteps < 1 || ckpt_every < 1) return fail(LME_EINVAL, "need nsteps >= 1 and ckpt_every >= 1");
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 > t0))
    return fail(LME_EINVAL, "need finite t0 < t1");
  if (h->n_ctrl < 1 || h->n_seg < 1)
    return fail(LME_EINVAL, "the gradient needs control terms and segments");
  if (!h->fn.empty())
    return fail(LME_ENOTSUP, "the gradient is taken with respect to piecewise-constant "
                "amplitudes; this handle has closed-form amplitudes");
  if (h->n_ctrl > 2) return fail(LME_ENOTSUP, "the gradient kernel takes at most 2 control terms");
  const double hstep = (t1 - t0) / nsteps;
  const double tl[2] = {t0, t1};
  std::vector<int32_t> tab;
  int rc = rk4_tables(h, 2, tl, nsteps, hstep, &tab);
  if (rc) return rc;
  int max_n2 = 0;
  for (auto &d : h->inst) max_n2 = std::max(max_n2, d.n * d.n);
  // Column layout (512 threads, at most 4 rows each; one control term, real
  // structure, the column kernels' operator shapes, adjoint of the same
  // shape): the column data of both operators in registers.  Otherwise the
  // row layout: 1024 threads (at most 4 elements each: twice the wavefronts
  // of the 512-thread configuration at the same packing), else 512 x 8.
  int wo = 0, nc = 0, nb = 0;
  bool col = h->n_ctrl == 1 && column_eligible(h, &wo, &nc, &nb) && nb == 1 && wo == 1 &&
             (nc == 2 || nc == 3) && real_structure(h) && column_fits(h, 512, 4, false);
  for (auto &d : h->inst)
    col = col && d.adj.wo == d.fwd.wo && d.adj.nc == d.fwd.nc && d.adj.wc == d.fwd.wc &&
          d.adj.nb == d.fwd.nb && d.adj.wb == d.fwd.wb;
  const int gl = h->tuning.grad_layout;
  if (gl == LME_LAYOUT_COLUMN && !col)
    return fail(LME_ENOTSUP, "the column layout of the gradient does not cover these operators");
  col = col && gl != LME_LAYOUT_ROW;
  int T = 1024, EPT = 0;
  if (col) {
    T = 512;
    EPT = 4;
  } else {
    for (int e : {1, 2, 4})
      if (!EPT && 1024 * e >= max_n2) EPT = e;
    if (!EPT && 512 * 8 >= max_n2) {
      T = 512;
      EPT = 8;
    }
  }
  if (!EPT)
    return fail(LME_ENOTSUP, "largest instance (%d elements) exceeds the gradient workgroup",
                max_n2);

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = ensure_device(h))) return rc;
  if ((rc = upload_tables(h, tab, s))) return rc;
  const int n_ck = (nsteps + ckpt_every - 1) / ckpt_every;
  const size_t ck_bytes = (size_t)n_ck * h->state_elems * 16;
  const size_t sb_bytes = (size_t)4 * ckpt_every * h->state_elems * 16;
  if (h->d_ckpt.bytes < ck_bytes + sb_bytes) {
    h->d_ckpt.release();
    hipError_t e = hipMalloc(&h->d_ckpt.p, ck_bytes + sb_bytes);
    if (e != hipSuccess) {
      h->d_ckpt.p = nullptr;
      return fail(LME_ENOMEM, "hipMalloc(checkpoints, %zu B) failed", ck_bytes + sb_bytes);
    }
    h->d_ckpt.bytes = ck_bytes + sb_bytes;
  }
  Plan *plan;
  if ((rc = plan_packs(h, T, EPT, 2, T * EPT, col ? 1 : 0, 2, &plan))) return rc;
  lme::GradArgs a;
  std::memset(&a, 0, sizeof a);
  a.packs = static_cast<const PackDesc *>(plan->d_packs.p);
  a.order = static_cast<const int32_t *>(plan->d_order.p);
  a.inst = static_cast<const InstDesc *>(h->d_inst.p);
  a.ops = static_cast<const uint8_t *>(h->d_ops.p);
  a.adj = static_cast<const uint8_t *>(h->d_adj.p);
  a.u = u_dev ? u_dev : static_cast<const double *>(h->d_u.p);
  a.n_ctrl = h->n_ctrl;
  a.n_seg = h->n_seg;
  a.seg_of_step = static_cast<const int32_t *>(h->d_steps.p);
  a.nsteps = nsteps;
  a.ckpt_every = ckpt_every;
  a.h = hstep;
  a.state_elems = h->state_elems;
  a.rho0 = static_cast<const double *>(rho0_dev);
  a.O = static_cast<const double *>(O_dev);
  a.ckpt = static_cast<double *>(h->d_ckpt.p);
  a.stages = reinterpret_cast<double *>(static_cast<uint8_t *>(h->d_ckpt.p) + ck_bytes);
  a.cost = cost_dev;
  a.grad = grad_dev;
  hipError_t e = col ? lme_internal_launch_grad_col(T, EPT, wo, nc, &a, (int)plan->packs.size(),
                                                    plan->max_lds, s)
                     : lme_internal_launch_grad(T, EPT, h->n_ctrl, &a, (int)plan->packs.size(),
                                                plan->max_lds, s);
  if (e != hipSuccess) return hip_fail(e, "launch gradient");
  return LME_OK;
}

extern "C" int lme_cost_grad(lme_handle h, int32_t nsteps, int32_t ckpt_every, double t0,
                             double t1, const void *rho0_dev, const void *O_dev,
                             const double *u_dev, double *cost_dev, double *grad_dev,
                             void *stream) {
  try {
    return cost_grad_impl(h, nsteps, ckpt_every, t0, t1, rho0_dev, O_dev, u_dev, cost_dev,
                          grad_dev, stream);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
extern "C" int lme_get_tuning(lme_handle h, lme_tuning *t) {
  if (!h || !t) return fail(LME_EINVAL, "handle and tuning must not be NULL");
  *t = h->tuning;
  t->apply_cap = h->apply_cap;
  t->apply_lds_kb = h->apply_lds_kb;
  t->apply_block = h->apply_block;
  t->apply_path = h->apply_path;
  return LME_OK;
}

extern "C" int lme_set_tuning(lme_handle h, const lme_tuning *t) {
  if (!h || !t) return fail(LME_EINVAL, "handle and tuning must not be NULL");
  if (t->rk4_layout < LME_LAYOUT_AUTO || t->rk4_layout > LME_LAYOUT_COLUMN)
    return fail(LME_EINVAL, "unknown layout %d", t->rk4_layout);
  if (t->rk4_block != 0 && t->rk4_block != 256 && t->rk4_block != 512 && t->rk4_block != 768 &&
      t->rk4_block != 1024)
    return fail(LME_EINVAL, "block must be 0, 256, 512, 768 or 1024");
  if (t->apply_cap != 0 && (t->apply_cap < 256 || t->apply_cap > 65536))
    return fail(LME_EINVAL, "apply_cap must be 0 or in [256, 65536]");
  if (t->apply_lds_kb != 0 && (t->apply_lds_kb < 16 || t->apply_lds_kb > 160))
    return fail(LME_EINVAL, "apply_lds_kb must be 0 or in [16, 160]");
  if (t->apply_block != 0 && t->apply_block != 256 && t->apply_block != 512 &&
      t->apply_block != 1024)
    return fail(LME_EINVAL, "apply_block must be 0, 256, 512 or 1024");
  if (t->apply_path != 0 && t->apply_path != 1)
    return fail(LME_EINVAL, "apply_path must be 0 or 1");
  if (t->herm_layout < LME_LAYOUT_AUTO || t->herm_layout > LME_LAYOUT_COLUMN)
    return fail(LME_EINVAL, "unknown layout %d", t->herm_layout);
  if (t->herm_block != 0 && t->herm_block != 256 && t->herm_block != 512 &&
      t->herm_block != 768 && t->herm_block != 1024)
    return fail(LME_EINVAL, "herm_block must be 0, 256, 512, 768 or 1024");
  if (t->grad_layout < LME_LAYOUT_AUTO || t->grad_layout > LME_LAYOUT_COLUMN)
    return fail(LME_EINVAL, "unknown layout %d", t->grad_layout);
  h->tuning = *t;
  h->apply_cap = t->apply_cap ? t->apply_cap : 4096;
  h->tuning.apply_cap = h->apply_cap;
  h->apply_lds_kb = t->apply_lds_kb;
  h->apply_block = t->apply_block ? t->apply_block : 1024;
  h->tuning.apply_block = h->apply_block;
  h->apply_path = t->apply_path;
  return LME_OK;
}

namespace {
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};
}  // namespace

static int autotune_impl(lme_handle h, const lme_options *opt, const void *rho0_dev, void *stream,
                         lme_tuning *result) {
  if (!h || !opt || !rho0_dev) return fail(LME_EINVAL, "handle, options and rho0 are required");
  if (opt->method != LME_RK4 || opt->nsteps < 1)
    return fail(LME_EINVAL, "the autotuner times RK4 runs: method RK4 and nsteps >= 1");
  int rc = ensure_device(h);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  DevBuf out;
  hipError_t e = hipMalloc(&out.p, (size_t)h->state_elems * 16);
  if (e != hipSuccess) {
    out.p = nullptr;
    return fail(LME_ENOMEM, "autotune scratch");
  }
  out.bytes = (size_t)h->state_elems * 16;
  EventPair ev;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
    return hip_fail(e, "hipEventCreate");
  auto time_ms = [&](auto &&launch, int reps, float *ms) -> int {
    int r = launch();  // warm-up (plans, uploads)
    if (r) return r;
    (void)hipEventRecord(ev.a, s);
    for (int i = 0; i < reps && !r; ++i) r = launch();
    (void)hipEventRecord(ev.b, s);
    hipError_t x = hipEventSynchronize(ev.b);
    if (r) return r;
    if (x != hipSuccess) return hip_fail(x, "hipEventSynchronize");
    (void)hipEventElapsedTime(ms, ev.a, ev.b);
    *ms /= reps;
    return LME_OK;
  };

  // RK4: layout x block on a trial of the caller's step size
  const int trial = std::min(opt->nsteps, 40);
  const double tl[2] = {0.0, 0.01 * trial};  // cost per step does not depend on h
  const lme_tuning saved = h->tuning;
  const bool herm = opt->hermitian == 1;
  h->tuning.rk4_block = 0;  // no tuned defaults while trying
  h->tuning.herm_block = 0;
  struct Cand { int layout, block; };
  const Cand cands[] = {{LME_LAYOUT_COLUMN, 1024}, {LME_LAYOUT_COLUMN, 768},
                        {LME_LAYOUT_COLUMN, 512}, {LME_LAYOUT_ROW, 256},
                        {LME_LAYOUT_ROW, 512}, {LME_LAYOUT_ROW, 1024}};
  float best = -1.0f;
  Cand win = {0, 0};
  for (const Cand &c : cands) {
    lme_options o = *opt;
    o.nsteps = trial;
    o.layout = c.layout;
    o.block = c.block;
    float ms = 0.0f;
    rc = time_ms([&]() { return evolve_impl(h, &o, 2, tl, rho0_dev, nullptr, nullptr, nullptr,
                                            out.p, nullptr, nullptr, stream, false); }, 2, &ms);
    if (rc == LME_ENOTSUP || rc == LME_EINVAL || rc == LME_EGRID) continue;  // not eligible
    if (rc) {
      h->tuning = saved;
      return rc;
    }
    if (best < 0.0f || ms < best) {
      best = ms;
      win = c;
    }
  }
  if (best < 0.0f) {
    h->tuning = saved;
    return fail(LME_ENOTSUP, "no RK4 configuration fits this batch");
  }
  h->tuning.rk4_block = saved.rk4_block;
  h->tuning.herm_block = saved.herm_block;
  if (herm) {
    h->tuning.herm_layout = win.layout;
    h->tuning.herm_block = win.block;
    h->tuning.herm_ms_per_step = best / trial;
  } else {
    h->tuning.rk4_layout = win.layout;
    h->tuning.rk4_block = win.block;
    h->tuning.rk4_ms_per_step = best / trial;
  }

  // application: workgroup size and LDS budget (column layout; smaller
  // budgets put more workgroups on a CU, whose loads then overlap the others'
  // arithmetic) or pack size (row layout)
  struct ACand { int path, block, kb, cap; };
  std::vector<ACand> acs;
  int wo, nc, nb;
  if (column_eligible(h, &wo, &nc, &nb)) {
    acs.push_back({0, h->apply_block, h->apply_lds_kb, h->apply_cap});
    for (int block : {1024, 512})
      for (int kb : {0, 80, 40}) acs.push_back({1, block, kb, h->apply_cap});
  } else {
    for (int cap : {512, 2048, 8192})
      acs.push_back({h->apply_path, h->apply_block, h->apply_lds_kb, cap});
  }
  float best_a = -1.0f;
  ACand best_c = {h->apply_path, h->apply_block, h->apply_lds_kb, h->apply_cap};
  for (const ACand &c : acs) {
    h->apply_path = c.path;
    h->apply_block = c.block;
    h->apply_lds_kb = c.kb;
    h->apply_cap = c.cap;
    float us = 0.0f;
    rc = time_ms([&]() { return apply_impl(h, LME_FORM_OPERATOR, 0, 0.0, nullptr, rho0_dev,
                                           out.p, stream); }, 5, &us);
    if (rc == LME_ENOTSUP) continue;
    if (rc) return rc;
    if (best_a < 0.0f || us < best_a) {
      best_a = us;
      best_c = c;
    }
  }
  h->apply_path = best_c.path;
  h->apply_block = best_c.block;
  h->apply_lds_kb = best_c.kb;
  h->apply_cap = best_c.cap;
  h->tuning.apply_path = best_c.path;
  h->tuning.apply_block = best_c.block;
  h->tuning.apply_cap = best_c.cap;
  h->tuning.apply_lds_kb = best_c.kb;
  h->tuning.apply_us = best_a * 1e3;
  if (result) *result = h->tuning;
  return LME_OK;
}

extern "C" int lme_autotune(lme_handle h, const lme_options *opt, const void *rho0_dev,
                            void *stream, lme_tuning *result) {
  try {
    return autotune_impl(h, opt, rho0_dev, stream, result);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

// ---------------------------------------------------------------------------
// Monte-Carlo wave-function trajectories (Sec. 3.2)
// ---------------------------------------------------------------------------
extern "C" int lme_internal_mc_rows(int *rows, int *max_threads, int cap);
extern "C" int lme_internal_mc_lds_bytes(int T, int P, int n);
extern "C" hipError_t lme_internal_launch_mc(int R, const lme::McArgs *a, int grid, int lds,
                                             hipStream_t s);
extern "C" hipError_t lme_internal_launch_mc_average(const double *ex_traj, double *expect,
                                                     int n_traj, int per, hipStream_t s);

struct lme_mc_ctx {
  int n = 0, wo = 0, nc = 0, wc = 0, ne = 0, we = 0;
  lme::McLayout L;
  std::vector<uint8_t> tabs;   // operator tables (layout lme::mc_layout), host image
  int device = 0, lds_limit = 0, n_cu = 0;
  bool on_device = false;
  DevBuf d_tabs, d_out, d_ex, d_vbuf;
  std::vector<int32_t> out_key;
};

static int mc_ensure_device(lme_mc_ctx *h) {
  hipError_t e;
  if (h->on_device) {
    e = hipSetDevice(h->device);
    return e == hipSuccess ? LME_OK : hip_fail(e, "hipSetDevice");
  }
  if ((e = hipGetDevice(&h->device)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipDeviceGetAttribute(&h->lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                 h->device)) != hipSuccess)
    return hip_fail(e, "hipDeviceGetAttribute(LDS)");
  if ((e = hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device)) !=
      hipSuccess)
    return hip_fail(e, "hipDeviceGetAttribute(CUs)");
  int rc = h->d_tabs.upload(h->tabs.data(), h->tabs.size(), "Monte-Carlo operator tables");
  if (rc) return rc;
  h->on_device = true;
  return LME_OK;
}

static int mc_create_impl(const lme_csr *H, int32_t n_c, const lme_csr *C, int32_t n_e,
                          const lme_csr *E, lme_mc_handle *out) {
  if (!out) return fail(LME_EINVAL, "out is NULL");
  *out = nullptr;
  if (!H) return fail(LME_EINVAL, "H is NULL");
  const int n = H->n;
  if (n < 1) return fail(LME_EINVAL, "n must be >= 1");
  if (n > lme::kMcMaxDim) return fail(LME_ENOTSUP, "n=%d exceeds %d", n, lme::kMcMaxDim);
  if (n_c < 0 || (n_c > 0 && !C)) return fail(LME_EINVAL, "bad collapse-operator list");
  if (n_c > lme::kMcMaxNC) return fail(LME_ENOTSUP, "at most %d collapse operators", lme::kMcMaxNC);
  if (n_e < 0 || (n_e > 0 && !E)) return fail(LME_EINVAL, "bad expectation-operator list");
  Sparse Hs;
  int rc = check_csr(H, n, "H", 0, &Hs);
  if (rc) return rc;
  std::vector<Sparse> Cs(n_c), Es(n_e);
  for (int k = 0; k < n_c; ++k)
    if ((rc = check_csr(&C[k], n, "C", 0, &Cs[k]))) return rc;
  for (int m = 0; m < n_e; ++m)
    if ((rc = check_csr(&E[m], n, "E", 0, &Es[m]))) return rc;
  // A = -i H_eff = -i H - 1/2 sum_k C_k^+ C_k  (Eq. (heff), hbar = 1)
  Sparse A(n);
  A.axpy(cd(0.0, -1.0), Hs);
  for (auto &c : Cs) A.axpy(cd(-0.5, 0.0), dag_times_self(c));
  A.finalize();
  std::unique_ptr<lme_mc_ctx> h(new (std::nothrow) lme_mc_ctx);
  if (!h) return fail(LME_ENOMEM, "out of host memory");
  h->n = n;
  h->wo = A.width_offdiag();
  h->nc = n_c;
  h->ne = n_e;
  for (auto &c : Cs) h->wc = std::max(h->wc, c.width());
  for (auto &m : Es) h->we = std::max(h->we, m.width());
  if (h->wo > lme::kMaxWidth || h->wc > lme::kMaxWidth || h->we > lme::kMaxWidth)
    return fail(LME_ENOTSUP, "an operator row has more than %d non-zeros", lme::kMaxWidth);
  h->L = lme::mc_layout(n, h->wo, h->nc, h->wc, h->ne, h->we);
  if (h->L.bytes > (int64_t)1 << 31) return fail(LME_ENOTSUP, "operator tables exceed 2 GiB");
  h->tabs.assign((size_t)h->L.bytes, 0);
  // (an empty table, e.g. A with no off-diagonal entries, copies nothing)
  auto put_c = [&](int64_t off, const std::vector<cd> &v) {
    if (!v.empty()) std::memcpy(h->tabs.data() + off, v.data(), v.size() * sizeof(cd));
  };
  auto put_i = [&](int64_t off, const std::vector<int32_t> &v) {
    if (!v.empty()) std::memcpy(h->tabs.data() + off, v.data(), v.size() * sizeof(int32_t));
  };
  put_c(h->L.offD, diag_of(A));
  Ell o = to_ell(A, h->wo, true);
  put_c(h->L.offOval, o.val);
  put_i(h->L.offOcol, o.col);
  for (int k = 0; k < n_c; ++k) {
    Ell e = to_ell(Cs[k], h->wc, false);
    put_c(h->L.offJval + 16LL * k * h->wc * n, e.val);
    put_i(h->L.offJcol + 4LL * k * h->wc * n, e.col);
  }
  for (int m = 0; m < n_e; ++m) {
    Ell e = to_ell(Es[m], h->we, false);
    put_c(h->L.offEval + 16LL * m * h->we * n, e.val);
    put_i(h->L.offEcol + 4LL * m * h->we * n, e.col);
  }
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) == hipSuccess && n_dev > 0) {
    if ((rc = mc_ensure_device(h.get()))) return rc;
  } else {
    (void)hipGetLastError();
  }
  *out = h.release();
  return LME_OK;
}

extern "C" int lme_mc_create(const lme_csr *H, int32_t n_c, const lme_csr *C, int32_t n_e,
                             const lme_csr *E, lme_mc_handle *out) {
  try {
    return mc_create_impl(H, n_c, C, n_e, E, out);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

extern "C" void lme_mc_destroy(lme_mc_handle h) { delete h; }

// Work decomposition: G threads (a power of two) per trajectory with R rows
// each (R a compiled row count, G * P within the kernel's largest workgroup),
// about five rows per thread; P trajectories per workgroup, bounded by LDS,
// enough workgroups for every CU when the trajectories allow it.
static int mc_plan(const lme_mc_ctx *h, int n_traj, int *R, int *G, int *P) {
  int rows[32], maxT[32];
  const int nr = lme_internal_mc_rows(rows, maxT, 32);
  const int n = h->n;
  *R = 0;
  for (int i = 0; i < nr && !*R; ++i) {
    if (rows[i] < std::min(n, 5)) continue;
    int g = 1;
    while (g * rows[i] < n) g <<= 1;
    // the smallest power of two covering n with rows[i] rows per thread
    if (g <= maxT[i]) {
      *R = rows[i];
      *G = g;
      int Pmax = maxT[i] / g;
      while (Pmax > 0 && lme_internal_mc_lds_bytes(Pmax * g, Pmax, n) > h->lds_limit) --Pmax;
      if (Pmax < 1) {
        *R = 0;
        continue;
      }
      const int want = std::max((64 + g - 1) / g, (n_traj + 2 * h->n_cu - 1) / (2 * h->n_cu));
      *P = std::max(1, std::min({Pmax, want, n_traj}));
    }
  }
  if (!*R)
    return fail(LME_ENOTSUP, "dimension %d does not fit the Monte-Carlo workgroup (%d B LDS)", n,
                h->lds_limit);
  return LME_OK;
}

static int mc_evolve_impl(lme_mc_handle h, int32_t n_t, const double *tlist, int32_t nsteps,
                          const void *psi0_dev, int32_t n_traj, const double *draws_dev,
                          int32_t max_jumps, void *expect_dev, void *expect_traj_dev,
                          int32_t *n_jumps_dev, double *jump_t_dev, int32_t *jump_op_dev,
                          int32_t *status_dev, void *stream) {
  if (!h) return fail(LME_EINVAL, "handle is NULL");
  int rc = check_times(n_t, tlist);
  if (rc) return rc;
  if (!psi0_dev || !draws_dev) return fail(LME_EINVAL, "psi0 and draws are required");
  if (n_traj < 1) return fail(LME_EINVAL, "n_traj must be >= 1");
  if (max_jumps < 0) return fail(LME_EINVAL, "max_jumps must be >= 0");
  if ((int64_t)n_traj * (max_jumps + 1) * 2 > ((int64_t)1 << 31))
    return fail(LME_ENOTSUP, "the draws table exceeds 2^31 numbers");
  if (n_t > 1 && nsteps < 1) return fail(LME_EINVAL, "need nsteps >= 1");
  const int32_t ns = n_t > 1 ? nsteps : 0;
  const double hstep = n_t > 1 ? (tlist[n_t - 1] - tlist[0]) / nsteps : 0.0;
  std::vector<int32_t> out_step(n_t, 0);
  for (int k = 1; k < n_t; ++k) {
    const long m = grid_index(tlist[k], tlist[0], hstep);
    if (m < 0 || m > ns)
      return fail(LME_EGRID, "output time %.17g is not on the RK4 grid (h = %.17g)", tlist[k],
                  hstep);
    out_step[k] = (int32_t)m;
  }
  if (n_t > 1 && out_step[n_t - 1] != ns)
    return fail(LME_EGRID, "last output time is not the end of the grid");
  // validation done: from here on the device is used
  if ((rc = mc_ensure_device(h))) return rc;
  int R = 0, G = 0, P = 0;
  if ((rc = mc_plan(h, n_traj, &R, &G, &P))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (out_step != h->out_key || !h->d_out.p) {
    if ((rc = h->d_out.upload(out_step.data(), out_step.size() * sizeof(int32_t), "output steps")))
      return rc;
    h->out_key = out_step;
  }
  const int n_packs = (n_traj + P - 1) / P;
  const int grid = std::min(n_packs, 8 * std::max(1, h->n_cu));
  const size_t per = (size_t)h->ne * n_t;
  auto ensure = [&](DevBuf &b, size_t bytes, const char *what) -> int {
    if (b.bytes >= bytes && b.p) return LME_OK;
    b.release();
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      b.p = nullptr;
      return fail(LME_ENOMEM, "hipMalloc(%s, %zu B) failed", what, bytes);
    }
    b.bytes = bytes;
    return LME_OK;
  };
  double *ex_traj = static_cast<double *>(expect_traj_dev);
  if (!ex_traj && per > 0) {
    if ((rc = ensure(h->d_ex, std::max<size_t>(16, 16 * per * n_traj), "trajectory outputs")))
      return rc;
    ex_traj = static_cast<double *>(h->d_ex.p);
  }
  if ((rc = ensure(h->d_vbuf, (size_t)grid * 64 * P * h->n, "jump scratch"))) return rc;

  const uint8_t *tb = static_cast<const uint8_t *>(h->d_tabs.p);
  lme::McArgs a;
  std::memset(&a, 0, sizeof a);
  a.n = h->n;
  a.wo = h->wo;
  a.nc = h->nc;
  a.wc = h->wc;
  a.ne = h->ne;
  a.we = h->we;
  a.G = G;
  a.P = P;
  a.n_traj = n_traj;
  a.n_t = n_t;
  a.nsteps = ns;
  a.max_jumps = max_jumps;
  a.t0 = tlist[0];
  a.h = hstep;
  a.D = reinterpret_cast<const double *>(tb + h->L.offD);
  a.Oval = reinterpret_cast<const double *>(tb + h->L.offOval);
  a.Ocol = reinterpret_cast<const int32_t *>(tb + h->L.offOcol);
  a.Jval = reinterpret_cast<const double *>(tb + h->L.offJval);
  a.Jcol = reinterpret_cast<const int32_t *>(tb + h->L.offJcol);
  a.Eval = reinterpret_cast<const double *>(tb + h->L.offEval);
  a.Ecol = reinterpret_cast<const int32_t *>(tb + h->L.offEcol);
  a.out_step = static_cast<const int32_t *>(h->d_out.p);
  a.psi0 = static_cast<const double *>(psi0_dev);
  a.draws = draws_dev;
  a.ex_traj = ex_traj;
  a.n_jumps = n_jumps_dev;
  a.jump_t = jump_t_dev;
  a.jump_op = jump_op_dev;
  a.status = status_dev;
  a.vbuf = static_cast<double *>(h->d_vbuf.p);
  const int lds = lme_internal_mc_lds_bytes(P * G, P, h->n);
  hipError_t e = lme_internal_launch_mc(R, &a, grid, lds, s);
  if (e != hipSuccess) return hip_fail(e, "launch Monte-Carlo kernel");
  if (expect_dev && per > 0) {
    e = lme_internal_launch_mc_average(ex_traj, static_cast<double *>(expect_dev), n_traj,
                                       (int)per, s);
    if (e != hipSuccess) return hip_fail(e, "launch trajectory average");
  }
  return LME_OK;
}

extern "C" int lme_mc_evolve(lme_mc_handle h, int32_t n_t, const double *tlist, int32_t nsteps,
                             const void *psi0_dev, int32_t n_traj, const double *draws_dev,
                             int32_t max_jumps, void *expect_dev, void *expect_traj_dev,
                             int32_t *n_jumps_dev, double *jump_t_dev, int32_t *jump_op_dev,
                             int32_t *status_dev, void *stream) {
  try {
    return mc_evolve_impl(h, n_t, tlist, nsteps, psi0_dev, n_traj, draws_dev, max_jumps,
                          expect_dev, expect_traj_dev, n_jumps_dev, jump_t_dev, jump_op_dev,
                          status_dev, stream);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

// ---------------------------------------------------------------------------
// Two-time correlation functions (quantum regression theorem)
// ---------------------------------------------------------------------------
extern "C" hipError_t lme_internal_launch_left_mul(int n_inst, int n_t, int wB, int64_t state_elems,
                                                   const int64_t *off, const int32_t *dims,
                                                   const int64_t *boff, const double *Bval,
                                                   const int32_t *Bcol, const double *states,
                                                   double *sigma, hipStream_t s);
extern "C" hipError_t lme_internal_launch_corr_status(const int32_t *st1, const int32_t *st2,
                                                      int32_t *status, int n_inst, int n_t,
                                                      hipStream_t s);

// The batch with instance b repeated reps[b] times (copies share the
// operators), the copies of b packed one after another, instances in order.
static std::unique_ptr<lme_ctx> make_replica(const lme_ctx *h, const std::vector<int> &reps) {
  std::unique_ptr<lme_ctx> r(new lme_ctx);
  int64_t total = 0;
  for (int b = 0; b < h->n_inst; ++b) total += reps[b];
  r->n_inst = (int32_t)total;
  r->n_ctrl = h->n_ctrl;
  r->n_e = h->n_e;
  r->n_seg = 0;
  r->ops = h->ops;
  r->adj = h->adj;
  r->eops = h->eops;
  r->inst.resize((size_t)r->n_inst);
  r->offsets.resize((size_t)r->n_inst);
  r->dims.resize((size_t)r->n_inst);
  int q = 0;
  int64_t off = 0;
  for (int b = 0; b < h->n_inst; ++b)
    for (int i = 0; i < reps[b]; ++i, ++q) {
      InstDesc d = h->inst[b];
      d.rho_off = off;
      off += (int64_t)d.n * d.n;
      r->inst[q] = d;
      r->offsets[q] = d.rho_off;
      r->dims[q] = d.n;
    }
  r->state_elems = off;
  return r;
}

static std::unique_ptr<lme_ctx> make_replica(const lme_ctx *h, int reps) {
  return make_replica(h, std::vector<int>((size_t)h->n_inst, reps));
}

struct CorrCache {
  std::unique_ptr<lme_ctx> rep;
  int reps = 0;
  DevBuf d_states, d_sigma, d_st1, d_st2, d_boff, d_bval, d_bcol, d_off, d_dims;
  // propagators: the batch repeated n_b^2 times, workspace of two
  // propagator sets, their offsets, the product's tile list
  std::unique_ptr<lme_ctx> prep;
  DevBuf d_p0, d_p1, d_pst, d_off4, d_first, d_tiles, d_diff;
  int n_tiles = 0;
};

static void corr_cache_free(void *p) { delete static_cast<CorrCache *>(p); }
static CorrCache *corr_cache(lme_ctx *h);

static int correlation_impl(lme_handle h, const lme_options *opt, int32_t n_t,
                            const double *tlist, int32_t n_tau, const double *taulist,
                            int32_t tau_nsteps, const lme_csr *B, const void *rho0_dev,
                            void *corr_dev, int32_t *status_dev, void *stream) {
  if (!h) return fail(LME_EINVAL, "handle is NULL");
  if (!opt) return fail(LME_EINVAL, "options are NULL");
  if (!rho0_dev || !corr_dev) return fail(LME_EINVAL, "rho0 and corr are required");
  if (!B) return fail(LME_EINVAL, "B is NULL");
  if (h->n_ctrl > 0)
    return fail(LME_ENOTSUP, "correlation functions need a time-independent generator (no "
                "control terms)");
  if (h->n_e < 1) return fail(LME_EINVAL, "correlation functions need expectation operators");
  if (opt->method != LME_RK4) return fail(LME_ENOTSUP, "correlation functions use fixed-step RK4");
  int rc = check_times(n_tau, taulist);
  if (rc) return rc;
  if (taulist[0] != 0.0) return fail(LME_EINVAL, "taulist must start at 0");
  if (n_tau > 1 && tau_nsteps < 1) return fail(LME_EINVAL, "need tau_nsteps >= 1");
  if ((int64_t)h->n_inst * n_t > (int64_t)1 << 30)
    return fail(LME_ENOTSUP, "too many (instance, time) pairs");
  // B as ELL per instance
  int wB = 0;
  std::vector<Sparse> Bs((size_t)h->n_inst);
  for (int b = 0; b < h->n_inst; ++b) {
    if ((rc = check_csr(&B[b], h->dims[b], "B", b, &Bs[b]))) return rc;
    wB = std::max(wB, Bs[b].width());
  }
  wB = std::max(wB, 1);
  std::vector<int64_t> boff((size_t)h->n_inst);
  std::vector<cd> bval;
  std::vector<int32_t> bcol;
  for (int b = 0; b < h->n_inst; ++b) {
    boff[b] = (int64_t)bval.size();
    Ell e = to_ell(Bs[b], wB, false);
    bval.insert(bval.end(), e.val.begin(), e.val.end());
    bcol.insert(bcol.end(), e.col.begin(), e.col.end());
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if ((rc = ensure_device(h))) return rc;
  CorrCache *cc = corr_cache(h);
  if (cc->reps != n_t || !cc->rep) {
    cc->rep = make_replica(h, n_t);
    cc->reps = n_t;
  }
  lme_ctx *rep = cc->rep.get();
  auto ensure = [&](DevBuf &buf, size_t bytes, const char *what) -> int {
    if (buf.p && buf.bytes >= bytes) return LME_OK;
    buf.release();
    hipError_t e = hipMalloc(&buf.p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
      buf.p = nullptr;
      return fail(LME_ENOMEM, "hipMalloc(%s, %zu B) failed", what, bytes);
    }
    buf.bytes = std::max<size_t>(bytes, 16);
    return LME_OK;
  };
  const size_t sbytes = (size_t)n_t * h->state_elems * 16;
  if ((rc = ensure(cc->d_states, sbytes, "states at the first times"))) return rc;
  if ((rc = ensure(cc->d_sigma, sbytes, "B rho(t)"))) return rc;
  if ((rc = ensure(cc->d_st1, 4 * (size_t)h->n_inst, "status"))) return rc;
  if ((rc = ensure(cc->d_st2, 4 * (size_t)h->n_inst * n_t, "status"))) return rc;
  if ((rc = cc->d_boff.upload(boff.data(), boff.size() * 8, "B offsets"))) return rc;
  if ((rc = cc->d_bval.upload(bval.data(), bval.size() * 16, "B values"))) return rc;
  if ((rc = cc->d_bcol.upload(bcol.data(), bcol.size() * 4, "B columns"))) return rc;
  if ((rc = cc->d_off.upload(h->offsets.data(), h->offsets.size() * 8, "offsets"))) return rc;
  if ((rc = cc->d_dims.upload(h->dims.data(), h->dims.size() * 4, "dims"))) return rc;
  // 1. rho(t_i) for every first time
  lme_options o1 = *opt;
  if ((rc = evolve_impl(h, &o1, n_t, tlist, rho0_dev, nullptr, nullptr, cc->d_states.p, nullptr,
                        nullptr, static_cast<int32_t *>(cc->d_st1.p), stream, false)))
    return rc;
  // 2. sigma = B rho(t_i), packed as the replicated batch
  hipError_t e = lme_internal_launch_left_mul(
      h->n_inst, n_t, wB, h->state_elems, static_cast<const int64_t *>(cc->d_off.p),
      static_cast<const int32_t *>(cc->d_dims.p), static_cast<const int64_t *>(cc->d_boff.p),
      static_cast<const double *>(cc->d_bval.p), static_cast<const int32_t *>(cc->d_bcol.p),
      static_cast<const double *>(cc->d_states.p), static_cast<double *>(cc->d_sigma.p), s);
  if (e != hipSuccess) return hip_fail(e, "launch B rho(t)");
  // 3. Tr(E_m V(tau_j) sigma) for every (instance, first time); sigma is not
  // Hermitian, so the general kernels run
  lme_options o2 = *opt;
  o2.nsteps = tau_nsteps;
  o2.hermitian = 0;
  o2.path = LME_PATH_AUTO;
  if ((rc = evolve_impl(rep, &o2, n_tau, taulist, cc->d_sigma.p, nullptr, corr_dev, nullptr,
                        nullptr, nullptr, static_cast<int32_t *>(cc->d_st2.p), stream, false)))
    return rc;
  if (status_dev) {
    e = lme_internal_launch_corr_status(static_cast<const int32_t *>(cc->d_st1.p),
                                        static_cast<const int32_t *>(cc->d_st2.p), status_dev,
                                        h->n_inst, n_t, s);
    if (e != hipSuccess) return hip_fail(e, "launch correlation status");
  }
  return LME_OK;
}

extern "C" int lme_correlation(lme_handle h, const lme_options *opt, int32_t n_t,
                               const double *tlist, int32_t n_tau, const double *taulist,
                               int32_t tau_nsteps, const lme_csr *B, const void *rho0_dev,
                               void *corr_dev, int32_t *status_dev, void *stream) {
  try {
    return correlation_impl(h, opt, n_t, tlist, n_tau, taulist, tau_nsteps, B, rho0_dev,
                            corr_dev, status_dev, stream);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

// ---------------------------------------------------------------------------
// Propagators and the steady state of repeated propagation
// ---------------------------------------------------------------------------
extern "C" hipError_t lme_internal_launch_prop_hbasis(double *U, const int64_t *off4,
                                                      const int32_t *dims, int n_inst,
                                                      hipStream_t s);
extern "C" hipError_t lme_internal_launch_prop_combine(double *U, const int64_t *off4,
                                                       const int32_t *dims, int n_inst,
                                                       hipStream_t s);
extern "C" hipError_t lme_internal_launch_zgemm(const void *tiles, int n_tiles, const int64_t *off4,
                                                const int32_t *dims, const double *A,
                                                const double *B, double *C, hipStream_t s);
extern "C" hipError_t lme_internal_launch_prop_norm_diff(double *Un, const double *Uo,
                                                         const int64_t *off4, const int32_t *dims,
                                                         int n_inst, int64_t max_block,
                                                         double *tau, void *dm, hipStream_t s);
extern "C" hipError_t lme_internal_launch_prop_column0(const double *U, const int64_t *off4,
                                                       const int32_t *dims, const int64_t *off2,
                                                       int n_inst, double *rho, hipStream_t s);
extern "C" hipError_t lme_internal_launch_range_status(const int32_t *st, const int64_t *first,
                                                       int32_t *status, int n_inst,
                                                       hipStream_t s);

static CorrCache *corr_cache(lme_ctx *h) {
  if (!h->corr) {
    h->corr = new CorrCache;
    h->corr_free = corr_cache_free;
  }
  return static_cast<CorrCache *>(h->corr);
}

static int dev_ensure(DevBuf &buf, size_t bytes, const char *what) {
  if (buf.p && buf.bytes >= bytes) return LME_OK;
  buf.release();
  hipError_t e = hipMalloc(&buf.p, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) {
    buf.p = nullptr;
    return fail(LME_ENOMEM, "hipMalloc(%s, %zu B) failed", what, bytes);
  }
  buf.bytes = std::max<size_t>(bytes, 16);
  return LME_OK;
}

// Offsets of the propagator blocks: off4[b] = sum_{b' < b} n_{b'}^4.
static std::vector<int64_t> prop_offsets(const lme_ctx *h, int64_t *total) {
  std::vector<int64_t> off4((size_t)h->n_inst + 1, 0);
  for (int b = 0; b < h->n_inst; ++b) {
    const int64_t N = (int64_t)h->dims[b] * h->dims[b];
    off4[b + 1] = off4[b] + N * N;
  }
  *total = off4[h->n_inst];
  return off4;
}

// U of every instance into U_dev (column-major blocks at off4).
static int propagator_run(lme_ctx *h, const lme_options *opt, double t0, double t1, void *U_dev,
                          int32_t *status_dev, hipStream_t s, void *stream) {
  int64_t total = 0;
  std::vector<int64_t> off4 = prop_offsets(h, &total);
  CorrCache *cc = corr_cache(h);
  if (!cc->prep) {
    std::vector<int> reps((size_t)h->n_inst);
    for (int b = 0; b < h->n_inst; ++b) reps[b] = h->dims[b] * h->dims[b];
    cc->prep = make_replica(h, reps);
  }
  int rc;
  if ((rc = cc->d_off4.upload(off4.data(), off4.size() * 8, "propagator offsets"))) return rc;
  if ((rc = cc->d_dims.upload(h->dims.data(), h->dims.size() * 4, "dims"))) return rc;
  std::vector<int64_t> first((size_t)h->n_inst + 1, 0);
  for (int b = 0; b < h->n_inst; ++b) first[b + 1] = first[b] + (int64_t)h->dims[b] * h->dims[b];
  if ((rc = cc->d_first.upload(first.data(), first.size() * 8, "replica ranges"))) return rc;
  if ((rc = dev_ensure(cc->d_p1, (size_t)total * 16, "basis matrices"))) return rc;
  if ((rc = dev_ensure(cc->d_pst, 4 * (size_t)first[h->n_inst], "status"))) return rc;
  // the n^2 Hermitian basis matrices (|a><a|, |a><b| + |b><a|,
  // i(|b><a| - |a><b|)) are evolved on the Hermitian kernels (each pair
  // {i, j} once), then combined into the columns of the |i><j| basis
  hipError_t e = lme_internal_launch_prop_hbasis(static_cast<double *>(cc->d_p1.p),
                                                 static_cast<const int64_t *>(cc->d_off4.p),
                                                 static_cast<const int32_t *>(cc->d_dims.p),
                                                 h->n_inst, s);
  if (e != hipSuccess) return hip_fail(e, "launch basis matrices");
  lme_options o = *opt;
  o.hermitian = 1;
  const double tl[2] = {t0, t1};
  if ((rc = evolve_impl(cc->prep.get(), &o, 2, tl, cc->d_p1.p, nullptr, nullptr, nullptr, U_dev,
                        nullptr, static_cast<int32_t *>(cc->d_pst.p), stream, false)))
    return rc;
  e = lme_internal_launch_prop_combine(static_cast<double *>(U_dev),
                                       static_cast<const int64_t *>(cc->d_off4.p),
                                       static_cast<const int32_t *>(cc->d_dims.p), h->n_inst, s);
  if (e != hipSuccess) return hip_fail(e, "launch propagator basis change");
  if (status_dev) {
    e = lme_internal_launch_range_status(static_cast<const int32_t *>(cc->d_pst.p),
                                         static_cast<const int64_t *>(cc->d_first.p), status_dev,
                                         h->n_inst, s);
    if (e != hipSuccess) return hip_fail(e, "launch propagator status");
  }
  return LME_OK;
}

static int prop_check(lme_ctx *h, const lme_options *opt, double t0, double t1) {
  if (!h) return fail(LME_EINVAL, "handle is NULL");
  if (!opt) return fail(LME_EINVAL, "options are NULL");
  if (h->n_ctrl > 0)
    return fail(LME_ENOTSUP, "propagators here are for time-independent generators (no control "
                "terms)");
  if (opt->method != LME_RK4) return fail(LME_ENOTSUP, "propagators use fixed-step RK4");
  if (opt->nsteps < 1) return fail(LME_EINVAL, "need nsteps >= 1");
  if (!std::isfinite(t0) || !std::isfinite(t1) || !(t1 > t0))
    return fail(LME_EINVAL, "need finite t1 > t0");
  for (int b = 0; b < h->n_inst; ++b)
    if (h->dims[b] > 128)
      return fail(LME_ENOTSUP, "instance %d: n = %d; propagators are formed for n <= 128", b,
                  h->dims[b]);
  return LME_OK;
}

extern "C" int lme_propagator(lme_handle h, const lme_options *opt, double t0, double t1,
                              void *U_dev, int32_t *status_dev, void *stream) {
  try {
    int rc = prop_check(h, opt, t0, t1);
    if (rc) return rc;
    if (!U_dev) return fail(LME_EINVAL, "U is NULL");
    if ((rc = ensure_device(h))) return rc;
    return propagator_run(h, opt, t0, t1, U_dev, status_dev, reinterpret_cast<hipStream_t>(stream),
                          stream);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}

static int steadystate_impl(lme_handle h, const lme_options *opt, double T, int32_t max_sq,
                            double tol, void *rho_dev, int32_t *status_dev, int32_t *squarings,
                            void *stream) {
  int rc = prop_check(h, opt, 0.0, T);
  if (rc) return rc;
  if (!rho_dev) return fail(LME_EINVAL, "rho_ss is NULL");
  if (max_sq < 0 || max_sq > 200) return fail(LME_EINVAL, "max_squarings must be in [0, 200]");
  if (!std::isfinite(tol) || tol < 0.0) return fail(LME_EINVAL, "tol must be finite, >= 0");
  if (tol == 0.0) tol = 1e-12;
  if ((rc = ensure_device(h))) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  CorrCache *cc = corr_cache(h);
  int64_t total = 0;
  std::vector<int64_t> off4 = prop_offsets(h, &total);
  if ((rc = dev_ensure(cc->d_p0, (size_t)total * 16, "propagators"))) return rc;
  if ((rc = propagator_run(h, opt, 0.0, T, cc->d_p0.p, nullptr, s, stream))) return rc;
  // tiles of the products: 64 x 64 per workgroup, every instance
  std::vector<int32_t> tiles;
  for (int b = 0; b < h->n_inst; ++b) {
    const int N = h->dims[b] * h->dims[b], nt = (N + 63) / 64;
    for (int i = 0; i < nt; ++i)
      for (int j = 0; j < nt; ++j) {
        tiles.push_back(b);
        tiles.push_back(i);
        tiles.push_back(j);
        tiles.push_back(0);
      }
  }
  if ((rc = cc->d_tiles.upload(tiles.data(), tiles.size() * 4, "product tiles"))) return rc;
  const int n_tiles = (int)(tiles.size() / 4);
  if ((rc = dev_ensure(cc->d_p1, (size_t)total * 16, "propagators"))) return rc;
  if ((rc = dev_ensure(cc->d_diff, 32 * (size_t)h->n_inst, "differences"))) return rc;
  std::vector<double> dm(2 * (size_t)h->n_inst);
  int64_t max_block = 0;
  for (int b = 0; b < h->n_inst; ++b) max_block = std::max(max_block, off4[b + 1] - off4[b]);
  std::vector<int32_t> st((size_t)h->n_inst, LME_EMAXSTEPS);
  double *P0 = static_cast<double *>(cc->d_p0.p), *P1 = static_cast<double *>(cc->d_p1.p);
  const int64_t *doff4 = static_cast<const int64_t *>(cc->d_off4.p);
  const int32_t *ddims = static_cast<const int32_t *>(cc->d_dims.p);
  double *diff = static_cast<double *>(cc->d_diff.p);
  int k = 0;
  for (; k < max_sq; ++k) {
    hipError_t e = lme_internal_launch_zgemm(cc->d_tiles.p, n_tiles, doff4, ddims, P0, P0, P1, s);
    if (e != hipSuccess) return hip_fail(e, "launch propagator product");
    // rescale to unit trace (rounding moves the eigenvalue 1 by ~1e-16, which
    // k squarings would raise to the power 2^k), then the change and size
    e = lme_internal_launch_prop_norm_diff(P1, P0, doff4, ddims, h->n_inst, max_block, diff,
                                           diff + 2 * h->n_inst, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dm.data(), diff + 2 * h->n_inst, dm.size() * 8, hipMemcpyDeviceToHost,
                         s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "propagator convergence check");
    std::swap(P0, P1);
    bool all = true;
    for (int b = 0; b < h->n_inst; ++b) {
      const double d = dm[2 * b], m = dm[2 * b + 1];
      if (!std::isfinite(d) || !std::isfinite(m)) st[b] = LME_ENONFINITE;
      else if (d <= tol * m) st[b] = LME_OK;
      else st[b] = LME_EMAXSTEPS;
      all = all && st[b] != LME_EMAXSTEPS;
    }
    if (all) {
      ++k;
      break;
    }
  }
  if (squarings) *squarings = k;
  std::vector<int64_t> off2(h->offsets.begin(), h->offsets.end());
  if ((rc = cc->d_off.upload(off2.data(), off2.size() * 8, "offsets"))) return rc;
  hipError_t e = lme_internal_launch_prop_column0(P0, doff4, ddims,
                                                  static_cast<const int64_t *>(cc->d_off.p),
                                                  h->n_inst, static_cast<double *>(rho_dev), s);
  if (e != hipSuccess) return hip_fail(e, "launch steady state");
  if (status_dev) {
    e = hipMemcpyAsync(status_dev, st.data(), st.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "steady-state status");
  }
  return LME_OK;
}

extern "C" int lme_steadystate(lme_handle h, const lme_options *opt, double T,
                               int32_t max_squarings, double tol, void *rho_ss_dev,
                               int32_t *status_dev, int32_t *squarings, void *stream) {
  try {
    return steadystate_impl(h, opt, T, max_squarings, tol, rho_ss_dev, status_dev, squarings,
                            stream);
  } catch (const std::bad_alloc &) {
    return fail(LME_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(LME_EINVAL, "unexpected host exception");
  }
}
