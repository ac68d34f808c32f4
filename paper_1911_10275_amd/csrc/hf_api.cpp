// C ABI of the Newton-step library: argument checking, host topology and
// layout construction, device allocation, and the GMRES / GMRES-IR / Newton
// drivers that sequence the device kernels.  Every arithmetic step of the
// Newton iteration runs in the HIP kernels; the host only orders them, reads
// back scalar reduction results and applies the Givens rotations of GMRES.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <set>
#include <stdexcept>

#include "hf_internal.h"

using namespace hf;

namespace {

hf_status fail(hf_ctx *ctx, hf_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, HF_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRY(call)                 \
  do {                            \
    hf_status s_ = (call);        \
    if (s_ != HF_OK) return s_;   \
  } while (0)

template <typename T>
hf_status dalloc(hf_ctx *ctx, T **p, int64_t n) {
  void *q = nullptr;
  size_t bytes = (size_t)std::max<int64_t>(n, 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess)
    return fail(ctx, HF_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  ctx->allocs.push_back(q);
  *p = (T *)q;
  return HF_OK;
}

template <typename T>
hf_status upload(hf_ctx *ctx, T **p, const std::vector<T> &v) {
  TRY(dalloc(ctx, p, (int64_t)v.size()));
  if (!v.empty())
    HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  return HF_OK;
}

bool all_finite(const double *x, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

KParams kparams(const hf_ctx *ctx) {
  KParams kp;
  kp.s = ctx->s;
  kp.m = ctx->m;
  const double E = ctx->mat.E, nu = ctx->mat.nu;
  kp.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  kp.G = E / (2.0 * (1.0 + nu));
  kp.sigma_c = ctx->mat.sigma_c;
  kp.delta_c = 2.0 * ctx->mat.G_c / ctx->mat.sigma_c;
  kp.mu = ctx->mat.mu;
  kp.dt = ctx->mat.dt;
  kp.b_stab = ctx->opt.b_stab;
  kp.s_p = ctx->s_p;
  kp.freeze_p = ctx->freeze_p;
  return kp;
}

hf_status check_ctx(hf_ctx *ctx, int need_stage) {
  if (!ctx) return HF_EINVAL;
  if (ctx->stage < need_stage)
    return fail(ctx, HF_ESTATE, "call out of order (stage " + std::to_string(ctx->stage) +
                                    ", needs " + std::to_string(need_stage) + ")");
  return HF_OK;
}

hf_status check_inst(hf_ctx *ctx, int32_t inst) {
  if (inst != 0) return fail(ctx, HF_EINVAL, "one instance per context: inst must be 0");
  return HF_OK;
}

hf_status sync_read(hf_ctx *ctx, int n) {
  HIPCHK(hipMemcpyAsync(ctx->red_h, ctx->red, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HF_OK;
}

// ---- profiling of kernel classes ------------------------------------------
enum ProfClass { P_ASM = 0, P_INV, P_SPMV64, P_SPMV32, P_PREC, P_ORTHO, P_NCLASS };

int take_event(hf_ctx *ctx) {
  if (ctx->ev_used == ctx->evpool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return -1;
    ctx->evpool.push_back(ev);
  }
  return (int)ctx->ev_used++;
}

struct ProfScope {
  hf_ctx *ctx;
  int cls, e0 = -1;
  ProfScope(hf_ctx *c, int k) : ctx(c), cls(k) {
    if (!ctx->opt.profile) return;
    e0 = take_event(ctx);
    if (e0 >= 0) (void)hipEventRecord(ctx->evpool[e0], ctx->stream);
  }
  ~ProfScope() {
    if (!ctx->opt.profile || e0 < 0) return;
    int e1 = take_event(ctx);
    if (e1 < 0) return;
    (void)hipEventRecord(ctx->evpool[e1], ctx->stream);
    ctx->ev_pending.push_back({cls, e0, e1});
  }
};

void resolve_profile(hf_ctx *ctx) {
  if (ctx->ev_pending.empty()) {
    ctx->ev_used = 0;
    return;
  }
  (void)hipStreamSynchronize(ctx->stream);
  double *ms[P_NCLASS] = {&ctx->prof.ms_assemble, &ctx->prof.ms_blockinv, &ctx->prof.ms_spmv64,
                          &ctx->prof.ms_spmv32, &ctx->prof.ms_precond, &ctx->prof.ms_ortho};
  int64_t *cnt[P_NCLASS] = {&ctx->prof.n_assemble, &ctx->prof.n_blockinv, &ctx->prof.n_spmv64,
                            &ctx->prof.n_spmv32, &ctx->prof.n_precond, &ctx->prof.n_ortho};
  for (const auto &pe : ctx->ev_pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, ctx->evpool[pe[1]], ctx->evpool[pe[2]]) == hipSuccess) {
      *ms[pe[0]] += t;
      *cnt[pe[0]] += 1;
    }
  }
  ctx->ev_pending.clear();
  ctx->ev_used = 0;
}

}  // namespace

// ===========================================================================
extern "C" void hf_default_options(hf_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = HF_FP64;
  o->gmres_m = 60;
  o->gmres_maxit = 20000;
  o->ir_maxit = 100;
  o->newton_maxit = 25;
  o->rtol = 1e-10;
  o->rtol_inner = 1e-2;
  o->newton_tol = 1e-10;
  o->b_stab = 10.0;
  o->p_cutoff = 0.0;
  o->cutoff_on = 0;
  o->device = 0;
  o->profile = 0;
  o->stream = nullptr;
}

static hf_status validate_options(hf_ctx *ctx, const hf_options &o) {
  if (o.precision != HF_FP64 && o.precision != HF_FP32_IR)
    return fail(ctx, HF_EINVAL, "precision must be HF_FP64 or HF_FP32_IR");
  if (o.gmres_m < 1 || o.gmres_m > kMaxKrylov - 1) return fail(ctx, HF_EINVAL, "gmres_m out of range 1..256");
  if (o.gmres_maxit < 1 || o.ir_maxit < 1 || o.newton_maxit < 1)
    return fail(ctx, HF_EINVAL, "iteration caps must be positive");
  if (!(o.rtol > 0 && o.rtol < 1) || !(o.rtol_inner > 0 && o.rtol_inner < 1) || !(o.newton_tol > 0))
    return fail(ctx, HF_EINVAL, "tolerances must lie in (0, 1)");
  if (!(o.b_stab > 0)) return fail(ctx, HF_EINVAL, "b_stab must be positive");
  return HF_OK;
}

extern "C" hf_status hf_create(const hf_options *opt, hf_ctx **out) {
  if (!out) return HF_EINVAL;
  *out = nullptr;
  hf_ctx *ctx = new (std::nothrow) hf_ctx();
  if (!ctx) return HF_ENOMEM;
  if (opt) ctx->opt = *opt; else hf_default_options(&ctx->opt);
  hf_status st = validate_options(ctx, ctx->opt);
  if (st != HF_OK) { delete ctx; return st; }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) { delete ctx; return HF_EDEVICE; }
  if (ctx->opt.device < 0 || ctx->opt.device >= ndev) { delete ctx; return HF_EINVAL; }
  if (hipSetDevice(ctx->opt.device) != hipSuccess) { delete ctx; return HF_EDEVICE; }
  if (ctx->opt.stream) {
    ctx->stream = (hipStream_t)ctx->opt.stream;
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) { delete ctx; return HF_EDEVICE; }
    ctx->own_stream = true;
  }
  if (hipHostMalloc((void **)&ctx->red_h, 4 * kMaxKrylov * sizeof(double)) != hipSuccess) {
    delete ctx;
    return HF_ENOMEM;
  }
  *out = ctx;
  return HF_OK;
}

extern "C" void hf_destroy(hf_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->opt.device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (void *p : ctx->allocs) (void)hipFree(p);
  if (ctx->red_h) (void)hipHostFree(ctx->red_h);
  for (hipEvent_t ev : ctx->evpool) (void)hipEventDestroy(ev);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

extern "C" const char *hf_last_error(const hf_ctx *ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

extern "C" hf_status hf_set_options(hf_ctx *ctx, const hf_options *opt) {
  if (!ctx || !opt) return HF_EINVAL;
  TRY(validate_options(ctx, *opt));
  if (opt->device != ctx->opt.device || opt->stream != ctx->opt.stream)
    return fail(ctx, HF_EINVAL, "device and stream are fixed at hf_create");
  ctx->opt = *opt;
  return HF_OK;
}

// ===========================================================================
// Mesh upload: interior faces, neighbours, clamped node copies
// ===========================================================================
extern "C" hf_status hf_upload_mesh(hf_ctx *ctx, int dim, int order, int64_t n_vert,
                                    const double *xyz, int64_t n_elem, const int32_t *elem_vert,
                                    const uint8_t *dirichlet_vert, int32_t *inst_out) {
  if (!ctx) return HF_EINVAL;
  if (ctx->stage != 0) return fail(ctx, HF_ESTATE, "one instance per context: mesh already uploaded");
  if (dim != 2 && dim != 3) return fail(ctx, HF_EINVAL, "dim must be 2 or 3");
  if (order != 1 && order != 2) return fail(ctx, HF_EINVAL, "order must be 1 or 2");
  if (n_vert <= 0 || n_elem <= 0 || !xyz || !elem_vert)
    return fail(ctx, HF_EINVAL, "empty mesh or null array");
  if (n_elem > (int64_t)INT32_MAX / 8) return fail(ctx, HF_EINVAL, "too many elements");
  if (!all_finite(xyz, n_vert * dim)) return fail(ctx, HF_ENONFINITE, "non-finite vertex coordinate");
  const int NF = dim + 1;
  for (int64_t i = 0; i < n_elem * NF; ++i)
    if (elem_vert[i] < 0 || elem_vert[i] >= n_vert) return fail(ctx, HF_EINVAL, "vertex id out of range");
  Sizes &s = ctx->s;
  s.dim = dim;
  s.order = order;
  s.nn = order == 1 ? dim + 1 : (dim + 1) * (dim + 2) / 2;
  s.bu = s.nn * dim;
  s.nnf = order == 1 ? dim : dim * (dim + 1) / 2;
  s.n_vert = n_vert;
  s.ne = n_elem;
  s.n_u = n_elem * s.bu;
  HostLayout &h = ctx->h;
  h.xyz.assign(xyz, xyz + n_vert * dim);
  h.elem.assign(elem_vert, elem_vert + n_elem * NF);
  h.dirichlet.assign(n_vert, 0);
  if (dirichlet_vert)
    for (int64_t v = 0; v < n_vert; ++v) h.dirichlet[v] = dirichlet_vert[v] ? 1 : 0;

  // all element faces keyed by sorted vertex ids
  struct FaceRec {
    std::array<int32_t, 3> key;
    int32_t e;
    int32_t lf;
  };
  std::vector<FaceRec> recs;
  recs.reserve(n_elem * NF);
  for (int64_t e = 0; e < n_elem; ++e)
    for (int lf = 0; lf < NF; ++lf) {
      FaceRec r{{-1, -1, -1}, (int32_t)e, lf};
      int k = 0;
      for (int c = 0; c < NF; ++c)
        if (c != lf) r.key[k++] = elem_vert[e * NF + c];
      std::sort(r.key.begin(), r.key.begin() + dim);
      if (r.key[0] == r.key[1] || (dim == 3 && r.key[1] == r.key[2]))
        return fail(ctx, HF_EINVAL, "degenerate element (repeated vertex)");
      recs.push_back(r);
    }
  std::sort(recs.begin(), recs.end(), [](const FaceRec &a, const FaceRec &b) {
    return a.key != b.key ? a.key < b.key : a.e < b.e;
  });
  h.nbr.assign(n_elem * NF, -1);
  h.fid.assign(n_elem * NF, -1);
  h.face_vert.clear();
  h.face_em.clear();
  h.face_ep.clear();
  h.face_lfm.clear();
  std::vector<std::array<int32_t, 3>> bfacets;
  for (size_t i = 0; i < recs.size();) {
    size_t j = i + 1;
    while (j < recs.size() && recs[j].key == recs[i].key) ++j;
    if (j - i > 2) return fail(ctx, HF_EINVAL, "non-manifold face (shared by more than two elements)");
    if (j - i == 1) {
      bfacets.push_back(recs[i].key);
    } else {
      const FaceRec &a = recs[i], &b = recs[i + 1];  // a.e < b.e: minus = a
      const int32_t f = (int32_t)h.face_em.size();
      for (int k = 0; k < dim; ++k) h.face_vert.push_back(a.key[k]);
      h.face_em.push_back(a.e);
      h.face_ep.push_back(b.e);
      h.face_lfm.push_back(a.lf);
      h.nbr[(int64_t)a.e * NF + a.lf] = b.e;
      h.nbr[(int64_t)b.e * NF + b.lf] = a.e;
      h.fid[(int64_t)a.e * NF + a.lf] = f;
      h.fid[(int64_t)b.e * NF + b.lf] = f;
    }
    i = j;
  }
  s.nf = (int64_t)h.face_em.size();
  h.fperm_m.assign(s.nf * dim, 0);
  h.fperm_p.assign(s.nf * dim, 0);
  for (int64_t f = 0; f < s.nf; ++f)
    for (int k = 0; k < dim; ++k) {
      const int32_t v = h.face_vert[f * dim + k];
      for (int c = 0; c < NF; ++c) {
        if (h.elem[(int64_t)h.face_em[f] * NF + c] == v) h.fperm_m[f * dim + k] = c;
        if (h.elem[(int64_t)h.face_ep[f] * NF + c] == v) h.fperm_p[f * dim + k] = c;
      }
    }
  // clamped node copies: nodes on boundary facets whose vertices are all flagged
  std::vector<uint8_t> cv(n_vert, 0);
  std::set<std::pair<int32_t, int32_t>> ce;
  for (const auto &k : bfacets) {
    bool all = true;
    for (int c = 0; c < dim; ++c) all = all && h.dirichlet[k[c]];
    if (!all) continue;
    for (int c = 0; c < dim; ++c) cv[k[c]] = 1;
    for (int a = 0; a < dim; ++a)
      for (int b = a + 1; b < dim; ++b) ce.insert({std::min(k[a], k[b]), std::max(k[a], k[b])});
  }
  static const int E2[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  static const int E3[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
  h.clamp.assign(n_elem, 0u);
  for (int64_t e = 0; e < n_elem; ++e) {
    uint32_t mask = 0;
    const int32_t *ev = &h.elem[e * NF];
    for (int a = 0; a < s.nn; ++a) {
      bool c;
      if (a < NF) {
        c = cv[ev[a]];
      } else {
        const int *ed = dim == 2 ? E2[a - NF] : E3[a - NF];
        int32_t x = ev[ed[0]], y = ev[ed[1]];
        c = ce.count({std::min(x, y), std::max(x, y)}) > 0;
      }
      if (c)
        for (int i = 0; i < dim; ++i) mask |= 1u << (a * dim + i);
    }
    h.clamp[e] = mask;
  }
  // quadrature rules
  Rule fr = simplex_rule(dim - 1, order + 1);
  Rule vr = simplex_rule(dim, order);
  double wsum = 0.0;
  for (double w : fr.w) wsum += w;
  RuleTables &rt = ctx->rules;
  std::memset(&rt, 0, sizeof(rt));
  rt.nqf = fr.nq();
  rt.nqv = vr.nq();
  for (int q = 0; q < rt.nqf; ++q) {
    double sum = 0.0;
    for (int k = 0; k < dim - 1; ++k) {
      rt.fq_mu[q][k + 1] = fr.pts[q * (dim - 1) + k];
      sum += fr.pts[q * (dim - 1) + k];
    }
    rt.fq_mu[q][0] = 1.0 - sum;
    rt.fq_w[q] = fr.w[q] / wsum;
  }
  for (int q = 0; q < rt.nqv; ++q) {
    double sum = 0.0;
    for (int k = 0; k < dim; ++k) {
      rt.vq_lam[q][k + 1] = vr.pts[q * dim + k];
      sum += vr.pts[q * dim + k];
    }
    rt.vq_lam[q][0] = 1.0 - sum;
    rt.vq_w[q] = vr.w[q];
  }
  s.nqf = rt.nqf;
  s.nqv = rt.nqv;
  h.qp_state.assign(s.nf * s.nqf, 0);
  h.beta.assign(s.nf, 0);
  ctx->stage = 1;
  if (inst_out) *inst_out = 0;
  return HF_OK;
}

extern "C" hf_status hf_get_faces(hf_ctx *ctx, int32_t inst, int64_t *n_face, int32_t *face_vert,
                                  int32_t *face_elem, int32_t *nq_face) {
  TRY(check_ctx(ctx, 1));
  TRY(check_inst(ctx, inst));
  if (n_face) *n_face = ctx->s.nf;
  if (nq_face) *nq_face = ctx->s.nqf;
  if (face_vert) std::memcpy(face_vert, ctx->h.face_vert.data(), ctx->h.face_vert.size() * 4);
  if (face_elem)
    for (int64_t f = 0; f < ctx->s.nf; ++f) {
      face_elem[2 * f] = ctx->h.face_em[f];
      face_elem[2 * f + 1] = ctx->h.face_ep[f];
    }
  return HF_OK;
}

extern "C" hf_status hf_upload_interfaces(hf_ctx *ctx, int32_t inst, const uint8_t *qp_state,
                                          const uint8_t *beta) {
  TRY(check_ctx(ctx, 1));
  TRY(check_inst(ctx, inst));
  if (ctx->stage >= 2) return fail(ctx, HF_ESTATE, "interfaces are fixed after hf_finalize");
  const int64_t n = ctx->s.nf * ctx->s.nqf;
  if (qp_state) {
    for (int64_t i = 0; i < n; ++i)
      if (qp_state[i] > 2) return fail(ctx, HF_EINVAL, "interface state must be 0, 1 or 2");
    ctx->h.qp_state.assign(qp_state, qp_state + n);
  }
  if (beta) {
    for (int64_t f = 0; f < ctx->s.nf; ++f)
      if (beta[f] > 1) return fail(ctx, HF_EINVAL, "beta must be 0 or 1");
    ctx->h.beta.assign(beta, beta + ctx->s.nf);
  }
  return HF_OK;
}

extern "C" hf_status hf_set_material(hf_ctx *ctx, int32_t inst, const hf_material *mat) {
  TRY(check_ctx(ctx, 1));
  TRY(check_inst(ctx, inst));
  if (!mat) return fail(ctx, HF_EINVAL, "null material");
  if (!(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->sigma_c > 0) ||
      !(mat->G_c > 0) || !(mat->mu > 0) || !(mat->dt > 0))
    return fail(ctx, HF_EINVAL, "material: need E, sigma_c, G_c, mu, dt > 0 and -1 < nu < 0.5");
  ctx->mat.E = mat->E;
  ctx->mat.nu = mat->nu;
  ctx->mat.sigma_c = mat->sigma_c;
  ctx->mat.G_c = mat->G_c;
  ctx->mat.mu = mat->mu;
  ctx->mat.dt = mat->dt;
  ctx->mat.set = true;
  return HF_OK;
}

extern "C" hf_status hf_set_injection(hf_ctx *ctx, int32_t inst, int32_t n_src,
                                      const int64_t *vert, const double *q0) {
  TRY(check_ctx(ctx, 1));
  TRY(check_inst(ctx, inst));
  if (ctx->stage >= 2) return fail(ctx, HF_ESTATE, "injection is fixed after hf_finalize");
  if (n_src < 0 || (n_src > 0 && (!vert || !q0))) return fail(ctx, HF_EINVAL, "bad sources");
  for (int i = 0; i < n_src; ++i) {
    if (vert[i] < 0 || vert[i] >= ctx->s.n_vert) return fail(ctx, HF_EINVAL, "source vertex out of range");
    if (!std::isfinite(q0[i])) return fail(ctx, HF_ENONFINITE, "non-finite Q0");
  }
  ctx->h.src_vert.assign(vert, vert + n_src);
  ctx->h.src_q0.assign(q0, q0 + n_src);
  return HF_OK;
}

// ===========================================================================
// Finalize: pressure numbering, coupling strips, block pattern, device data
// ===========================================================================
extern "C" hf_status hf_finalize(hf_ctx *ctx) {
  TRY(check_ctx(ctx, 1));
  if (ctx->stage >= 2) return fail(ctx, HF_ESTATE, "already finalized");
  if (!ctx->mat.set) return fail(ctx, HF_ESTATE, "hf_set_material must precede hf_finalize");
  HIPCHK(hipSetDevice(ctx->opt.device));
  Sizes &s = ctx->s;
  HostLayout &h = ctx->h;
  const int dim = s.dim, NF = dim + 1, NNF = s.nnf, BU = s.bu;
  // ---- active faces and pressure nodes -----------------------------------
  h.act_face.clear();
  h.slot.assign(s.nf, -1);
  for (int64_t f = 0; f < s.nf; ++f)
    if (h.beta[f]) {
      h.slot[f] = (int32_t)h.act_face.size();
      h.act_face.push_back((int32_t)f);
    }
  s.n_act = (int64_t)h.act_face.size();
  static const int FE2[3][2] = {{0, 1}, {1, 2}, {2, 0}};
  auto face_keys = [&](int64_t f, std::vector<std::pair<int64_t, int64_t>> &ks) {
    ks.clear();
    const int32_t *fv = &h.face_vert[f * dim];
    for (int k = 0; k < dim; ++k) ks.push_back({fv[k], -1});
    if (s.order == 2) {
      const int ne_f = dim == 2 ? 1 : 3;
      for (int q = 0; q < ne_f; ++q) {
        int32_t a = fv[FE2[q][0]], b = fv[FE2[q][1]];
        ks.push_back({std::min(a, b), std::max(a, b)});
      }
    }
  };
  std::vector<std::pair<int64_t, int64_t>> vkeys, ekeys, ks;
  for (int32_t f : h.act_face) {
    face_keys(f, ks);
    for (auto &k : ks) (k.second < 0 ? vkeys : ekeys).push_back(k);
  }
  std::sort(vkeys.begin(), vkeys.end());
  vkeys.erase(std::unique(vkeys.begin(), vkeys.end()), vkeys.end());
  std::sort(ekeys.begin(), ekeys.end());
  ekeys.erase(std::unique(ekeys.begin(), ekeys.end()), ekeys.end());
  std::map<std::pair<int64_t, int64_t>, int32_t> pidx;
  h.pkeys.clear();
  for (auto &k : vkeys) { pidx[k] = (int32_t)pidx.size(); h.pkeys.push_back(k.first); h.pkeys.push_back(-1); }
  for (auto &k : ekeys) { pidx[k] = (int32_t)pidx.size(); h.pkeys.push_back(k.first); h.pkeys.push_back(k.second); }
  s.n_p = (int64_t)pidx.size();
  if (s.n_p > 4096) return fail(ctx, HF_EINVAL, "more than 4096 pressure nodes (dense pressure block limit)");
  h.face_pn.assign(s.n_act * NNF, -1);
  for (int64_t a = 0; a < s.n_act; ++a) {
    face_keys(h.act_face[a], ks);
    for (int k = 0; k < NNF; ++k) h.face_pn[a * NNF + k] = pidx.at(ks[k]);
  }
  std::vector<int32_t> src_node;
  for (size_t i = 0; i < h.src_vert.size(); ++i) {
    auto it = pidx.find({h.src_vert[i], -1});
    if (it == pidx.end()) return fail(ctx, HF_EINVAL, "injection vertex is not on a fluid face");
    src_node.push_back(it->second);
  }
  s.n_src = (int64_t)src_node.size();
  // ---- coupling strips: per element, the pressure nodes of its fluid faces
  std::vector<int64_t> sp_ptr(s.ne + 1, 0);
  std::vector<int32_t> sp_pnode, sp_elem, sp_se, strip_elems, fs_idx(s.ne * NF * NNF, -1);
  std::vector<int64_t> t_ptr(1, 0);
  for (int64_t e = 0; e < s.ne; ++e) {
    std::vector<int32_t> nodes;
    for (int lf = 0; lf < NF; ++lf) {
      int32_t f = h.fid[e * NF + lf];
      if (f < 0 || !h.beta[f]) continue;
      for (int k = 0; k < NNF; ++k) nodes.push_back(h.face_pn[(int64_t)h.slot[f] * NNF + k]);
    }
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    sp_ptr[e + 1] = sp_ptr[e] + (int64_t)nodes.size();
    if (!nodes.empty()) {
      if (nodes.size() > 32) return fail(ctx, HF_EINVAL, "coupling strip too long");
      const int32_t se = (int32_t)strip_elems.size();
      strip_elems.push_back((int32_t)e);
      t_ptr.push_back(t_ptr.back() + (int64_t)nodes.size() * (int64_t)nodes.size());
      for (int32_t nd : nodes) {
        sp_pnode.push_back(nd);
        sp_elem.push_back((int32_t)e);
        sp_se.push_back(se);
      }
      for (int lf = 0; lf < NF; ++lf) {
        int32_t f = h.fid[e * NF + lf];
        if (f < 0 || !h.beta[f]) continue;
        for (int k = 0; k < NNF; ++k) {
          int32_t nd = h.face_pn[(int64_t)h.slot[f] * NNF + k];
          int pos = (int)(std::lower_bound(nodes.begin(), nodes.end(), nd) - nodes.begin());
          fs_idx[(e * NF + lf) * NNF + k] = (int32_t)(sp_ptr[e] + pos);
        }
      }
    }
  }
  s.n_strip = (int64_t)sp_pnode.size();
  s.n_se = (int64_t)strip_elems.size();
  s.n_t = t_ptr.back();
  std::vector<int32_t> pc_ptr(s.n_p + 1, 0), pc_ent(s.n_strip);
  for (int32_t nd : sp_pnode) pc_ptr[nd + 1]++;
  for (int64_t i = 0; i < s.n_p; ++i) pc_ptr[i + 1] += pc_ptr[i];
  {
    std::vector<int32_t> fill(pc_ptr.begin(), pc_ptr.end() - 1);
    for (int64_t k = 0; k < s.n_strip; ++k) pc_ent[fill[sp_pnode[k]]++] = (int32_t)k;
  }
  std::vector<int32_t> pf_ptr(s.n_p + 1, 0), pf_fa, pf_k;
  {
    std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(s.n_p);
    for (int64_t a = 0; a < s.n_act; ++a)
      for (int k = 0; k < NNF; ++k) lists[h.face_pn[a * NNF + k]].push_back({(int32_t)a, k});
    for (int64_t i = 0; i < s.n_p; ++i) {
      pf_ptr[i + 1] = pf_ptr[i] + (int32_t)lists[i].size();
      for (auto &pr : lists[i]) {
        pf_fa.push_back(pr.first);
        pf_k.push_back(pr.second);
      }
    }
  }
  // ---- block pattern: diagonal, then one block per interior local face ----
  std::vector<int64_t> blk_ptr(s.ne + 1, 0);
  std::vector<int32_t> blk_col, blk_of(s.ne * NF, -1);
  for (int64_t e = 0; e < s.ne; ++e) {
    blk_col.push_back((int32_t)e);
    for (int lf = 0; lf < NF; ++lf) {
      int32_t nb = h.nbr[e * NF + lf];
      if (nb < 0) continue;
      blk_of[e * NF + lf] = (int32_t)blk_col.size();
      blk_col.push_back(nb);
    }
    blk_ptr[e + 1] = (int64_t)blk_col.size();
  }
  s.n_blocks = (int64_t)blk_col.size();
  std::vector<int64_t> ident_ptr(s.ne + 1);
  std::vector<int32_t> ident_col(s.ne);
  for (int64_t e = 0; e <= s.ne; ++e) ident_ptr[e] = e;
  for (int64_t e = 0; e < s.ne; ++e) ident_col[e] = (int32_t)e;
  // bounding box extent (fluid-row scale)
  double L = 0.0;
  for (int c = 0; c < dim; ++c) {
    double lo = 1e300, hi = -1e300;
    for (int64_t v = 0; v < s.n_vert; ++v) {
      lo = std::min(lo, h.xyz[v * dim + c]);
      hi = std::max(hi, h.xyz[v * dim + c]);
    }
    L = std::max(L, hi - lo);
  }
  h.bbox_L = L;

  // ---- device data -----------------------------------------------------------
  DevMesh &m = ctx->m;
  TRY(upload(ctx, &m.xyz, h.xyz));
  TRY(upload(ctx, &m.elem_vert, h.elem));
  TRY(dalloc(ctx, &m.gl, s.ne * NF * dim));
  TRY(dalloc(ctx, &m.detabs, s.ne));
  TRY(upload(ctx, &m.nbr, h.nbr));
  TRY(upload(ctx, &m.fid, h.fid));
  TRY(upload(ctx, &m.blk_of, blk_of));
  TRY(upload(ctx, &m.clamp, h.clamp));
  TRY(upload(ctx, &m.blk_ptr, blk_ptr));
  TRY(upload(ctx, &m.blk_col, blk_col));
  TRY(upload(ctx, &m.face_vert, h.face_vert));
  TRY(upload(ctx, &m.face_em, h.face_em));
  TRY(upload(ctx, &m.face_ep, h.face_ep));
  TRY(upload(ctx, &m.fperm_m, h.fperm_m));
  TRY(upload(ctx, &m.fperm_p, h.fperm_p));
  TRY(upload(ctx, &m.face_lfm, h.face_lfm));
  TRY(dalloc(ctx, &m.normal, s.nf * dim));
  TRY(dalloc(ctx, &m.area, s.nf));
  TRY(dalloc(ctx, &m.hf, s.nf));
  TRY(dalloc(ctx, &m.ginv, s.nf * (dim - 1) * (dim - 1)));
  TRY(upload(ctx, &m.qp_state, h.qp_state));
  TRY(upload(ctx, &m.beta, h.beta));
  TRY(upload(ctx, &m.slot, h.slot));
  TRY(upload(ctx, &m.act_face, h.act_face));
  TRY(upload(ctx, &m.face_pn, h.face_pn));
  TRY(upload(ctx, &m.fs_idx, fs_idx));
  TRY(upload(ctx, &m.sp_ptr, sp_ptr));
  TRY(upload(ctx, &m.sp_pnode, sp_pnode));
  TRY(upload(ctx, &m.sp_elem, sp_elem));
  TRY(upload(ctx, &m.sp_se, sp_se));
  TRY(upload(ctx, &m.pc_ptr, pc_ptr));
  TRY(upload(ctx, &m.pc_ent, pc_ent));
  TRY(upload(ctx, &m.pf_ptr, pf_ptr));
  TRY(upload(ctx, &m.pf_fa, pf_fa));
  TRY(upload(ctx, &m.pf_k, pf_k));
  TRY(upload(ctx, &m.src_node, src_node));
  TRY(upload(ctx, &m.src_q0, h.src_q0));
  TRY(upload(ctx, &m.strip_elems, strip_elems));
  TRY(upload(ctx, &m.t_ptr, t_ptr));
  TRY(upload(ctx, &m.ident_ptr, ident_ptr));
  TRY(upload(ctx, &m.ident_col, ident_col));
  // system and work buffers
  const int64_t N = s.N();
  TRY(dalloc(ctx, &ctx->xs, N));
  TRY(dalloc(ctx, &ctx->xs_save, N));
  TRY(dalloc(ctx, &ctx->xs_start, N));
  TRY(dalloc(ctx, &ctx->w_old, s.nf * s.nqf));
  TRY(dalloc(ctx, &ctx->w_tmp, s.nf * s.nqf));
  TRY(dalloc(ctx, &ctx->R, N));
  TRY(dalloc(ctx, &ctx->A, s.n_blocks * BU * BU));
  TRY(dalloc(ctx, &ctx->Bs, s.n_strip * BU));
  TRY(dalloc(ctx, &ctx->Cs, s.n_strip * BU));
  TRY(dalloc(ctx, &ctx->D, s.n_p * s.n_p));
  TRY(dalloc(ctx, &ctx->S, s.n_p * s.n_p));
  TRY(dalloc(ctx, &ctx->Sinv, s.n_p * s.n_p));
  TRY(dalloc(ctx, &ctx->Sinv32, s.n_p * s.n_p));
  TRY(dalloc(ctx, &ctx->T, s.n_t));
  TRY(dalloc(ctx, &ctx->inv, s.ne * BU * BU));
  TRY(dalloc(ctx, &ctx->flag, 4));
  TRY(dalloc(ctx, &ctx->dx, N));
  TRY(dalloc(ctx, &ctx->rhs, N));
  TRY(dalloc(ctx, &ctx->r64, N));
  TRY(dalloc(ctx, &ctx->t64, N));
  // reduction partials: the largest of (blocks x outputs) over every reduction
  const int64_t n_partial = std::max<int64_t>((int64_t)1024 * kMaxKrylov,
                                              (int64_t)ortho_blocks(N) * (kMaxKrylov + 1));
  TRY(dalloc(ctx, &ctx->partial, n_partial));
  TRY(dalloc(ctx, &ctx->red, 4 * kMaxKrylov));
  HIPCHK(hipMemsetAsync(ctx->xs, 0, N * sizeof(double), ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->w_old, 0, s.nf * s.nqf * sizeof(double), ctx->stream));
  HIPCHK(launch_set_rules(ctx->rules, ctx->stream));
  HIPCHK(launch_geometry(kparams(ctx), ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->stage = 2;
  return HF_OK;
}

extern "C" hf_status hf_get_sizes(hf_ctx *ctx, int32_t inst, hf_sizes *out) {
  TRY(check_ctx(ctx, 1));
  TRY(check_inst(ctx, inst));
  if (!out) return fail(ctx, HF_EINVAL, "null output");
  const Sizes &s = ctx->s;
  out->n_elem = s.ne;
  out->nodes_per_elem = s.nn;
  out->n_u = s.n_u;
  out->n_p = ctx->stage >= 2 ? s.n_p : 0;
  out->n_face = s.nf;
  out->n_blocks = ctx->stage >= 2 ? s.n_blocks : 0;
  out->dim = s.dim;
  out->order = s.order;
  out->nq_face = s.nqf;
  out->block_size = s.bu;
  return HF_OK;
}

extern "C" hf_status hf_get_pnodes(hf_ctx *ctx, int32_t inst, int64_t *keys) {
  TRY(check_ctx(ctx, 2));
  TRY(check_inst(ctx, inst));
  if (!keys && ctx->s.n_p) return fail(ctx, HF_EINVAL, "null output");
  if (ctx->s.n_p) std::memcpy(keys, ctx->h.pkeys.data(), ctx->h.pkeys.size() * sizeof(int64_t));
  return HF_OK;
}

// ===========================================================================
// State
// ===========================================================================
static hf_status update_fluid_scale(hf_ctx *ctx) {
  const double delta_c = 2.0 * ctx->mat.G_c / ctx->mat.sigma_c;
  double wmax = -1e300;
  if (ctx->s.n_act) {
    HIPCHK(launch_wmax(kparams(ctx), ctx->w_old, ctx->red, ctx->stream));
    TRY(sync_read(ctx, 1));
    wmax = ctx->red_h[0];
  }
  const double w_ref = std::max(wmax, 0.01 * delta_c);
  const double L = ctx->h.bbox_L;
  ctx->s_p = 12.0 * ctx->mat.mu * std::pow(L / w_ref, 3);
  return HF_OK;
}

extern "C" hf_status hf_set_state(hf_ctx *ctx, int32_t inst, const double *u, const double *p,
                                  const double *w_old) {
  TRY(check_ctx(ctx, 2));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  if (!u || (s.n_p && !p)) return fail(ctx, HF_EINVAL, "null state array");
  if (!all_finite(u, s.n_u) || (s.n_p && !all_finite(p, s.n_p)) ||
      (w_old && !all_finite(w_old, s.nf * s.nqf)))
    return fail(ctx, HF_ENONFINITE, "non-finite value in the state");
  HIPCHK(hipMemcpyAsync(ctx->xs, u, s.n_u * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  if (s.n_p)
    HIPCHK(hipMemcpyAsync(ctx->xs + s.n_u, p, s.n_p * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  if (w_old)
    HIPCHK(hipMemcpyAsync(ctx->w_old, w_old, s.nf * s.nqf * sizeof(double), hipMemcpyHostToDevice,
                          ctx->stream));
  TRY(update_fluid_scale(ctx));
  ctx->stage = 3;
  return HF_OK;
}

extern "C" hf_status hf_set_state_device(hf_ctx *ctx, int32_t inst, const double *u,
                                         const double *p, const double *w_old) {
  TRY(check_ctx(ctx, 2));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  if (!u || (s.n_p && !p)) return fail(ctx, HF_EINVAL, "null state array");
  HIPCHK(hipMemcpyAsync(ctx->xs, u, s.n_u * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (s.n_p)
    HIPCHK(hipMemcpyAsync(ctx->xs + s.n_u, p, s.n_p * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (w_old)
    HIPCHK(hipMemcpyAsync(ctx->w_old, w_old, s.nf * s.nqf * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->stream));
  HIPCHK(launch_norm2(ctx->xs, s.N(), ctx->partial, ctx->red, ctx->stream));
  TRY(sync_read(ctx, 1));
  if (!std::isfinite(ctx->red_h[0])) return fail(ctx, HF_ENONFINITE, "non-finite value in the state");
  TRY(update_fluid_scale(ctx));
  ctx->stage = 3;
  return HF_OK;
}

extern "C" hf_status hf_get_state(hf_ctx *ctx, int32_t inst, double *u, double *p, double *w,
                                  double *w_old) {
  TRY(check_ctx(ctx, 2));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  if (u) HIPCHK(hipMemcpyAsync(u, ctx->xs, s.n_u * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (p && s.n_p)
    HIPCHK(hipMemcpyAsync(p, ctx->xs + s.n_u, s.n_p * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (w) {
    HIPCHK(launch_set_rules(ctx->rules, ctx->stream));
    HIPCHK(launch_opening(kparams(ctx), ctx->xs, ctx->w_tmp, ctx->stream));
    HIPCHK(hipMemcpyAsync(w, ctx->w_tmp, s.nf * s.nqf * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  }
  if (w_old)
    HIPCHK(hipMemcpyAsync(w_old, ctx->w_old, s.nf * s.nqf * sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HF_OK;
}

extern "C" hf_status hf_get_state_device(hf_ctx *ctx, int32_t inst, double *u, double *p) {
  TRY(check_ctx(ctx, 2));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  if (u) HIPCHK(hipMemcpyAsync(u, ctx->xs, s.n_u * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  if (p && s.n_p)
    HIPCHK(hipMemcpyAsync(p, ctx->xs + s.n_u, s.n_p * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  return HF_OK;
}

// ===========================================================================
// Assembly
// ===========================================================================
static hf_status do_assemble(hf_ctx *ctx, double *res_norm) {
  const Sizes &s = ctx->s;
  KParams kp = kparams(ctx);
  HIPCHK(launch_set_rules(ctx->rules, ctx->stream));  // the rule tables are module-global
  {
    ProfScope ps(ctx, P_ASM);
    HIPCHK(launch_assemble(kp, ctx->xs, ctx->xs + s.n_u, ctx->w_old, ctx->A, ctx->R, ctx->Bs,
                           ctx->Cs, ctx->D, ctx->stream));
  }
  HIPCHK(launch_norm2(ctx->R, s.N(), ctx->partial, ctx->red, ctx->stream));
  TRY(sync_read(ctx, 1));
  const double rn = std::sqrt(ctx->red_h[0]);
  if (!std::isfinite(rn)) return fail(ctx, HF_ENONFINITE, "non-finite residual");
  if (res_norm) *res_norm = rn;
  ctx->have32 = false;
  return HF_OK;
}

extern "C" hf_status hf_assemble(hf_ctx *ctx, double *res_norm) {
  TRY(check_ctx(ctx, 3));
  HIPCHK(hipSetDevice(ctx->opt.device));
  TRY(do_assemble(ctx, res_norm));
  ctx->stage = std::max(ctx->stage, 4);
  return HF_OK;
}

// ===========================================================================
// Krylov solvers
// ===========================================================================
template <typename T>
struct Ops {
  const T *A, *Bs, *Cs, *D, *inv, *Sinv;
};

template <typename T>
static hf_status ensure_ws(hf_ctx *ctx, KrylovWs<T> &ws) {
  const int m = ctx->opt.gmres_m;
  const int64_t N = ctx->s.N();
  if (ws.V && ws.m >= m && ws.n == N) return HF_OK;
  TRY(dalloc(ctx, &ws.V, (int64_t)(m + 1) * N));
  TRY(dalloc(ctx, &ws.w, N));
  TRY(dalloc(ctx, &ws.z, N));
  TRY(dalloc(ctx, &ws.r, N));
  TRY(dalloc(ctx, &ws.t, N));
  TRY(dalloc(ctx, &ws.b, N));
  TRY(dalloc(ctx, &ws.x, N));
  ws.m = m;
  ws.n = N;
  return HF_OK;
}

template <typename T>
static hf_status apply_J(hf_ctx *ctx, const KParams &kp, const Ops<T> &op, const T *x, T *y) {
  if (sizeof(T) == 8) {
    ProfScope ps(ctx, P_SPMV64);
    HIPCHK(launch_spmv<T>(kp, op.A, op.Bs, op.Cs, op.D, x, y, ctx->stream));
  } else {
    ProfScope ps(ctx, P_SPMV32);
    HIPCHK(launch_spmv<T>(kp, op.A, op.Bs, op.Cs, op.D, x, y, ctx->stream));
  }
  return HF_OK;
}

template <typename T>
static hf_status apply_M(hf_ctx *ctx, const KParams &kp, const Ops<T> &op, const T *r, T *z) {
  ProfScope ps(ctx, P_PREC);
  HIPCHK(launch_precond<T>(kp, op.inv, op.Sinv, r, z, ctx->stream));
  return HF_OK;
}

template <typename T>
static hf_status vnorm(hf_ctx *ctx, const T *x, int64_t n, double &out) {
  HIPCHK(launch_mdot<T>(x, 0, 1, x, n, ctx->partial, ctx->red, ctx->stream));
  TRY(sync_read(ctx, 1));
  out = std::sqrt(ctx->red_h[0]);
  return HF_OK;
}

static bool trace_on() {
  static int on = -1;
  if (on < 0) {
    const char *e = std::getenv("HF_TRACE");
    on = (e && *e && *e != '0') ? 1 : 0;
  }
  return on == 1;
}

// HF_REORTH=0 disables the second Gram-Schmidt pass (experiments only)
static bool reorth_allowed() {
  static int on = -1;
  if (on < 0) {
    const char *e = std::getenv("HF_REORTH");
    on = (e && *e == '0') ? 0 : 1;
  }
  return on == 1;
}

// Right-preconditioned restarted GMRES(m) on J x = b in precision T with
// classical Gram-Schmidt applied twice.  x starts at 0.  A cycle ends when the
// recursive residual estimate reaches rtol ||b|| or after m steps; with
// explicit_check the residual b - J x is then recomputed and decides.
template <typename T>
static hf_status gmres(hf_ctx *ctx, const Ops<T> &op, KrylovWs<T> &ws, const T *b, T *x,
                       double rtol, int maxit, bool explicit_check, int &iters, int &restarts,
                       double &relres) {
  const KParams kp = kparams(ctx);
  const int64_t N = ctx->s.N();
  const int m = ctx->opt.gmres_m;
  HIPCHK(hipMemsetAsync(x, 0, N * sizeof(T), ctx->stream));
  double bnorm;
  TRY(vnorm<T>(ctx, b, N, bnorm));
  if (!std::isfinite(bnorm)) return fail(ctx, HF_ENONFINITE, "non-finite right-hand side");
  if (bnorm == 0.0) {
    relres = 0.0;
    return HF_OK;
  }
  HIPCHK(hipMemcpyAsync(ws.r, b, N * sizeof(T), hipMemcpyDeviceToDevice, ctx->stream));
  std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  double beta = bnorm;
  while (true) {
    if (explicit_check && beta <= rtol * bnorm) {
      relres = beta / bnorm;
      return HF_OK;
    }
    if (iters >= maxit) {
      relres = beta / bnorm;
      return fail(ctx, HF_ENOCONV, "GMRES reached its iteration cap");
    }
    HIPCHK(launch_scale_copy<T>(ws.r, 1.0 / beta, ws.V, N, ctx->stream));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      T *vj = ws.V + (int64_t)j * N;
      TRY(apply_M<T>(ctx, kp, op, vj, ws.z));
      TRY(apply_J<T>(ctx, kp, op, ws.z, ws.w));
      const int kk = j + 1;
      // classical Gram-Schmidt with the DGKS re-orthogonalisation test:
      // h = V^T w, w1 = w - V h; repeat once more when ||w1|| < ||w|| / sqrt(2)
      {
        ProfScope ps(ctx, P_ORTHO);
        HIPCHK(launch_proj<T>(ws.V, N, kk, ws.w, N, ctx->partial, ctx->red, ctx->stream));
        HIPCHK(launch_orth_update<T>(ws.V, N, kk, ctx->red, ws.w, N, ctx->partial,
                                     ctx->red + kk + 1, ctx->stream));
      }
      TRY(sync_read(ctx, kk + 2));
      ++iters;
      for (int i = 0; i < kk; ++i) H[i * m + j] = ctx->red_h[i];
      double hn = std::sqrt(ctx->red_h[kk + 1]);
      if (reorth_allowed() && hn < std::sqrt(0.5 * ctx->red_h[kk])) {
        {
          ProfScope ps(ctx, P_ORTHO);
          HIPCHK(launch_proj<T>(ws.V, N, kk, ws.w, N, ctx->partial, ctx->red, ctx->stream));
          HIPCHK(launch_orth_update<T>(ws.V, N, kk, ctx->red, ws.w, N, ctx->partial,
                                       ctx->red + kk + 1, ctx->stream));
        }
        TRY(sync_read(ctx, kk + 2));
        for (int i = 0; i < kk; ++i) H[i * m + j] += ctx->red_h[i];
        hn = std::sqrt(ctx->red_h[kk + 1]);
        ++ctx->n_reorth;
      }
      if (!std::isfinite(hn)) return fail(ctx, HF_ENONFINITE, "non-finite Krylov vector");
      H[kk * m + j] = hn;
      if (hn > 0.0) HIPCHK(launch_scale_copy<T>(ws.w, 1.0 / hn, ws.V + (int64_t)kk * N, N, ctx->stream));
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t;
      }
      const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = H[j * m + j] / den;
        sn[j] = H[(j + 1) * m + j] / den;
      }
      H[j * m + j] = cs[j] * H[j * m + j] + sn[j] * H[(j + 1) * m + j];
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      if (std::fabs(g[j + 1]) <= rtol * bnorm || iters >= maxit || hn == 0.0) break;
    }
    // y = H(1:k,1:k)^-1 g ; x += M^-1 V y
    for (int i = k - 1; i >= 0; --i) {
      double acc = g[i];
      for (int c = i + 1; c < k; ++c) acc -= H[i * m + c] * y[c];
      y[i] = acc / H[i * m + i];
    }
    std::memcpy(ctx->red_h, y.data(), k * sizeof(double));
    HIPCHK(hipMemcpyAsync(ctx->red, ctx->red_h, k * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(launch_combine<T>(ws.V, N, k, ctx->red, ws.t, N, ctx->stream));
    TRY(apply_M<T>(ctx, kp, op, ws.t, ws.z));
    HIPCHK(launch_axpy_t<T>(1.0, ws.z, x, N, ctx->stream));
    ++restarts;
    const double est = std::fabs(g[k]);
    if (!explicit_check && (est <= rtol * bnorm || iters >= maxit)) {
      HIPCHK(hipStreamSynchronize(ctx->stream));
      relres = est / bnorm;
      return HF_OK;
    }
    TRY(apply_J<T>(ctx, kp, op, x, ws.w));
    HIPCHK(launch_sub_t<T>(b, ws.w, ws.r, N, ctx->stream));
    TRY(vnorm<T>(ctx, ws.r, N, beta));
    if (!std::isfinite(beta)) return fail(ctx, HF_ENONFINITE, "non-finite residual in GMRES");
    if (trace_on())
      std::fprintf(stderr, "hf gmres(%s): it %d restart %d estimate %.3e true %.3e reorth %lld\n",
                   sizeof(T) == 8 ? "fp64" : "fp32", iters, restarts, est / bnorm, beta / bnorm,
                   (long long)ctx->n_reorth);
  }
}

static hf_status build_preconditioner(hf_ctx *ctx) {
  const Sizes &s = ctx->s;
  const KParams kp = kparams(ctx);
  const bool ir = ctx->opt.precision == HF_FP32_IR;
  if (ir && !ctx->inv32) {
    TRY(dalloc(ctx, &ctx->inv32, s.ne * s.bu * s.bu));
    TRY(dalloc(ctx, &ctx->A32, s.n_blocks * s.bu * s.bu));
    TRY(dalloc(ctx, &ctx->Bs32, s.n_strip * s.bu));
    TRY(dalloc(ctx, &ctx->Cs32, s.n_strip * s.bu));
    TRY(dalloc(ctx, &ctx->D32, s.n_p * s.n_p));
  }
  HIPCHK(hipMemsetAsync(ctx->flag, 0, sizeof(int), ctx->stream));
  {
    ProfScope ps(ctx, P_INV);
    HIPCHK(launch_blockinv(kp, ctx->A, ctx->inv, ir ? ctx->inv32 : nullptr, ctx->flag, ctx->stream));
  }
  HIPCHK(launch_schur(kp, ctx->inv, ctx->Bs, ctx->Cs, ctx->D, nullptr, ctx->T, ctx->S, ctx->Sinv,
                      ctx->Sinv32, ctx->flag, ctx->stream));
  if (ir) {
    HIPCHK(launch_convert(ctx->A, ctx->A32, s.n_blocks * s.bu * s.bu, ctx->stream));
    HIPCHK(launch_convert(ctx->Bs, ctx->Bs32, s.n_strip * s.bu, ctx->stream));
    HIPCHK(launch_convert(ctx->Cs, ctx->Cs32, s.n_strip * s.bu, ctx->stream));
    HIPCHK(launch_convert(ctx->D, ctx->D32, s.n_p * s.n_p, ctx->stream));
    ctx->have32 = true;
  }
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, ctx->flag, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (flag & 1) return fail(ctx, HF_ESINGULAR, "zero or non-finite pivot in an element block");
  if (flag & 2) return fail(ctx, HF_ESINGULAR, "zero or non-finite pivot in the pressure block");
  return HF_OK;
}

static hf_status do_solve(hf_ctx *ctx, hf_solve_stats *stats) {
  const auto t0 = std::chrono::steady_clock::now();
  const Sizes &s = ctx->s;
  const int64_t N = s.N();
  const KParams kp = kparams(ctx);
  hf_solve_stats st{};
  TRY(build_preconditioner(ctx));
  HIPCHK(launch_axpby(-1.0, ctx->R, 0.0, ctx->rhs, N, ctx->stream));  // b = -R
  hf_status status = HF_OK;
  if (ctx->opt.precision == HF_FP64) {
    TRY(ensure_ws<double>(ctx, ctx->k64));
    Ops<double> op{ctx->A, ctx->Bs, ctx->Cs, ctx->D, ctx->inv, ctx->Sinv};
    status = gmres<double>(ctx, op, ctx->k64, ctx->rhs, ctx->dx, ctx->opt.rtol, ctx->opt.gmres_maxit,
                           true, st.gmres_iters, st.restarts, st.true_relres);
  } else {
    TRY(ensure_ws<float>(ctx, ctx->k32));
    Ops<double> op64{ctx->A, ctx->Bs, ctx->Cs, ctx->D, ctx->inv, ctx->Sinv};
    Ops<float> op32{ctx->A32, ctx->Bs32, ctx->Cs32, ctx->D32, ctx->inv32, ctx->Sinv32};
    HIPCHK(hipMemsetAsync(ctx->dx, 0, N * sizeof(double), ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->r64, ctx->rhs, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    double bnorm;
    TRY(vnorm<double>(ctx, ctx->rhs, N, bnorm));
    if (!std::isfinite(bnorm)) return fail(ctx, HF_ENONFINITE, "non-finite right-hand side");
    st.true_relres = 0.0;
    const int cap = 20 * ctx->opt.gmres_m;
    if (bnorm > 0.0) {
      status = HF_ENOCONV;
      for (int outer = 0; outer < ctx->opt.ir_maxit; ++outer) {
        double rn;
        TRY(vnorm<double>(ctx, ctx->r64, N, rn));
        st.true_relres = rn / bnorm;
        if (!std::isfinite(rn)) return fail(ctx, HF_ENONFINITE, "non-finite refinement residual");
        if (rn <= ctx->opt.rtol * bnorm) {
          status = HF_OK;
          break;
        }
        if (st.gmres_iters >= ctx->opt.gmres_maxit) break;
        HIPCHK(launch_cast_scale(ctx->r64, 1.0 / rn, ctx->k32.b, N, ctx->stream));
        int inner_it = 0, inner_rs = 0;
        double est = 0.0;
        const int lim = std::min(cap, ctx->opt.gmres_maxit - st.gmres_iters);
        hf_status is = gmres<float>(ctx, op32, ctx->k32, ctx->k32.b, ctx->k32.x, ctx->opt.rtol_inner,
                                    lim, false, inner_it, inner_rs, est);
        if (is != HF_OK && is != HF_ENOCONV) return is;
        st.gmres_iters += inner_it;
        st.restarts += inner_rs;
        st.ir_steps += 1;
        HIPCHK(launch_cast_axpy(rn, ctx->k32.x, ctx->dx, N, ctx->stream));
        TRY(apply_J<double>(ctx, kp, op64, ctx->dx, ctx->t64));
        HIPCHK(launch_sub(ctx->rhs, ctx->t64, ctx->r64, N, ctx->stream));
      }
      if (status != HF_OK) fail(ctx, HF_ENOCONV, "GMRES-IR did not reach rtol within its caps");
    }
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return status;
}

extern "C" hf_status hf_solve(hf_ctx *ctx, hf_solve_stats *stats) {
  TRY(check_ctx(ctx, 4));
  HIPCHK(hipSetDevice(ctx->opt.device));
  TRY(do_solve(ctx, stats));
  ctx->stage = 5;
  return HF_OK;
}

// ===========================================================================
// Newton
// ===========================================================================
static hf_status do_newton_step(hf_ctx *ctx, hf_newton_stats *ns) {
  const Sizes &s = ctx->s;
  double rn = 0.0;
  TRY(do_assemble(ctx, &rn));
  ctx->stage = std::max(ctx->stage, 4);
  hf_solve_stats ls{};
  hf_status st = do_solve(ctx, &ls);
  if (ns) {
    ns->lin = ls;
    ns->res_norm = rn;
  }
  if (st != HF_OK) return st;  // state untouched
  HIPCHK(hipMemcpyAsync(ctx->xs_save, ctx->xs, s.N() * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(launch_newton_update(ctx->dx, ctx->xs, s.n_u, ctx->xs + s.n_u, s.n_p, ctx->opt.cutoff_on,
                              ctx->opt.p_cutoff, ctx->partial, ctx->red, ctx->stream));
  TRY(sync_read(ctx, 4));
  const double du = std::sqrt(ctx->red_h[0]), un = std::sqrt(ctx->red_h[1]);
  const double dp = std::sqrt(ctx->red_h[2]), pn = std::sqrt(ctx->red_h[3]);
  if (!std::isfinite(du) || !std::isfinite(un) || !std::isfinite(dp) || !std::isfinite(pn)) {
    HIPCHK(hipMemcpyAsync(ctx->xs, ctx->xs_save, s.N() * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return fail(ctx, HF_ENONFINITE, "non-finite Newton update");
  }
  const double ru = un > 0.0 ? du / un : du;
  const double rp = s.n_p ? (pn > 0.0 ? dp / pn : dp) : 0.0;
  if (ns) {
    ns->du_rel = ru;
    ns->dp_rel = rp;
    ns->iterations += 1;
    ns->converged = (ru <= ctx->opt.newton_tol && rp <= ctx->opt.newton_tol) ? 1 : 0;
  }
  ctx->stage = 3;
  return HF_OK;
}

extern "C" hf_status hf_newton_step(hf_ctx *ctx, hf_newton_stats *stats) {
  TRY(check_ctx(ctx, 3));
  HIPCHK(hipSetDevice(ctx->opt.device));
  hf_newton_stats ns{};
  hf_status st = do_newton_step(ctx, &ns);
  if (stats) *stats = ns;
  return st;
}

extern "C" hf_status hf_newton_solve(hf_ctx *ctx, hf_newton_stats *stats) {
  TRY(check_ctx(ctx, 3));
  HIPCHK(hipSetDevice(ctx->opt.device));
  const int64_t N = ctx->s.N();
  HIPCHK(hipMemcpyAsync(ctx->xs_start, ctx->xs, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  hf_newton_stats acc{};
  hf_status st = HF_OK;
  for (int k = 0; k < ctx->opt.newton_maxit; ++k) {
    hf_newton_stats one{};
    st = do_newton_step(ctx, &one);
    acc.lin.gmres_iters += one.lin.gmres_iters;
    acc.lin.ir_steps += one.lin.ir_steps;
    acc.lin.restarts += one.lin.restarts;
    acc.lin.true_relres = std::max(acc.lin.true_relres, one.lin.true_relres);
    acc.lin.seconds += one.lin.seconds;
    acc.du_rel = one.du_rel;
    acc.dp_rel = one.dp_rel;
    acc.res_norm = one.res_norm;
    acc.iterations += 1;
    if (st != HF_OK) break;
    if (one.converged) {
      acc.converged = 1;
      break;
    }
  }
  if (stats) *stats = acc;
  if (st != HF_OK || !acc.converged) {
    // restore the state at the start of the call
    HIPCHK(hipMemcpyAsync(ctx->xs, ctx->xs_start, N * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (st == HF_OK) st = fail(ctx, HF_ENOCONV, "Newton did not converge within newton_maxit");
    return st;
  }
  return HF_OK;
}

extern "C" hf_status hf_initial_guess(hf_ctx *ctx, double *p0_out) {
  TRY(check_ctx(ctx, 3));
  HIPCHK(hipSetDevice(ctx->opt.device));
  const Sizes &s = ctx->s;
  double q_total = 0.0;
  for (double q : ctx->h.src_q0) q_total += q;
  if (!s.n_p || q_total <= 0.0) {
    if (p0_out) *p0_out = 0.0;
    return HF_OK;  // nothing to predict: keep the state
  }
  // unit-pressure elastic response u1 with the pressure held fixed
  HIPCHK(hipMemsetAsync(ctx->xs, 0, s.n_u * sizeof(double), ctx->stream));
  HIPCHK(launch_fill(1.0, ctx->xs + s.n_u, s.n_p, ctx->stream));
  ctx->freeze_p = 1;
  hf_status st = do_assemble(ctx, nullptr);
  if (st == HF_OK) st = do_solve(ctx, nullptr);
  ctx->freeze_p = 0;
  if (st != HF_OK) return st;
  HIPCHK(hipMemcpyAsync(ctx->xs, ctx->dx, s.n_u * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(launch_set_rules(ctx->rules, ctx->stream));
  HIPCHK(launch_fluid_volume(kparams(ctx), ctx->xs, ctx->partial, ctx->red, ctx->stream));
  TRY(sync_read(ctx, 1));
  const double V1 = ctx->red_h[0];
  if (!(V1 > 0.0) || !std::isfinite(V1))
    return fail(ctx, HF_ENONFINITE, "unit-pressure crack volume is not positive");
  const double p0 = q_total * ctx->mat.dt / V1;
  HIPCHK(launch_axpby(0.0, ctx->dx, p0, ctx->xs, s.n_u, ctx->stream));  // u0 = p0 u1
  HIPCHK(launch_fill(p0, ctx->xs + s.n_u, s.n_p, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (p0_out) *p0_out = p0;
  ctx->stage = 3;
  return HF_OK;
}

extern "C" hf_status hf_end_load_step(hf_ctx *ctx) {
  TRY(check_ctx(ctx, 3));
  HIPCHK(hipSetDevice(ctx->opt.device));
  HIPCHK(launch_set_rules(ctx->rules, ctx->stream));
  HIPCHK(launch_opening(kparams(ctx), ctx->xs, ctx->w_old, ctx->stream));
  TRY(update_fluid_scale(ctx));
  ctx->stage = 3;
  return HF_OK;
}

// ===========================================================================
// Inspection hooks
// ===========================================================================
extern "C" hf_status hf_get_residual(hf_ctx *ctx, int32_t inst, double *R_u, double *R_p) {
  TRY(check_ctx(ctx, 4));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  if (R_u) HIPCHK(hipMemcpyAsync(R_u, ctx->R, s.n_u * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (R_p && s.n_p)
    HIPCHK(hipMemcpyAsync(R_p, ctx->R + s.n_u, s.n_p * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HF_OK;
}

extern "C" hf_status hf_get_block_rows(hf_ctx *ctx, int32_t inst, int64_t n_rows,
                                       const int32_t *elems, int32_t *cols, double *blocks) {
  TRY(check_ctx(ctx, 4));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  const int NF = s.dim + 1, BU = s.bu, NS = s.dim + 2;
  if (n_rows < 0 || (n_rows && (!elems || !cols || !blocks))) return fail(ctx, HF_EINVAL, "bad arguments");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // host copy of the block positions
  std::vector<double> buf(BU * BU);
  for (int64_t i = 0; i < n_rows; ++i) {
    const int32_t e = elems[i];
    if (e < 0 || e >= s.ne) return fail(ctx, HF_EINVAL, "element out of range");
    for (int slot = 0; slot < NS; ++slot) {
      int64_t blk = -1;
      int32_t col = -1;
      if (slot == 0) {
        // diagonal block is the first of the row
        int64_t bp = 0;
        HIPCHK(hipMemcpy(&bp, ctx->m.blk_ptr + e, sizeof(int64_t), hipMemcpyDeviceToHost));
        blk = bp;
        col = e;
      } else if (slot - 1 < NF && ctx->h.nbr[(int64_t)e * NF + slot - 1] >= 0) {
        int32_t b = 0;
        HIPCHK(hipMemcpy(&b, ctx->m.blk_of + (int64_t)e * NF + slot - 1, sizeof(int32_t), hipMemcpyDeviceToHost));
        blk = b;
        col = ctx->h.nbr[(int64_t)e * NF + slot - 1];
      }
      cols[i * NS + slot] = col;
      double *out = blocks + (i * NS + slot) * BU * BU;
      if (blk < 0) {
        std::fill(out, out + BU * BU, 0.0);
        continue;
      }
      HIPCHK(hipMemcpy(buf.data(), ctx->A + blk * BU * BU, BU * BU * sizeof(double), hipMemcpyDeviceToHost));
      for (int c = 0; c < BU; ++c)
        for (int r = 0; r < BU; ++r) out[r * BU + c] = buf[c * BU + r];
    }
  }
  return HF_OK;
}

extern "C" hf_status hf_get_coupling(hf_ctx *ctx, int32_t inst, double *B, double *C, double *D) {
  TRY(check_ctx(ctx, 4));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  const int BU = s.bu;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::vector<double> bs(s.n_strip * BU), cs(s.n_strip * BU);
  std::vector<int64_t> sp_ptr(s.ne + 1);
  std::vector<int32_t> sp_pnode(s.n_strip);
  HIPCHK(hipMemcpy(bs.data(), ctx->Bs, bs.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(cs.data(), ctx->Cs, cs.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(sp_ptr.data(), ctx->m.sp_ptr, sp_ptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  if (s.n_strip)
    HIPCHK(hipMemcpy(sp_pnode.data(), ctx->m.sp_pnode, sp_pnode.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (B) std::fill(B, B + s.n_u * s.n_p, 0.0);
  if (C) std::fill(C, C + s.n_p * s.n_u, 0.0);
  for (int64_t e = 0; e < s.ne; ++e)
    for (int64_t k = sp_ptr[e]; k < sp_ptr[e + 1]; ++k)
      for (int r = 0; r < BU; ++r) {
        if (B) B[(e * BU + r) * s.n_p + sp_pnode[k]] = bs[k * BU + r];
        if (C) C[sp_pnode[k] * s.n_u + e * BU + r] = cs[k * BU + r];
      }
  if (D && s.n_p) HIPCHK(hipMemcpy(D, ctx->D, s.n_p * s.n_p * sizeof(double), hipMemcpyDeviceToHost));
  return HF_OK;
}

extern "C" hf_status hf_get_increment(hf_ctx *ctx, int32_t inst, double *du, double *dp) {
  TRY(check_ctx(ctx, 3));
  TRY(check_inst(ctx, inst));
  const Sizes &s = ctx->s;
  if (du) HIPCHK(hipMemcpyAsync(du, ctx->dx, s.n_u * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  if (dp && s.n_p)
    HIPCHK(hipMemcpyAsync(dp, ctx->dx + s.n_u, s.n_p * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HF_OK;
}

extern "C" hf_status hf_apply_jacobian(hf_ctx *ctx, int precision, const void *x, void *y) {
  TRY(check_ctx(ctx, 4));
  if (!x || !y) return fail(ctx, HF_EINVAL, "null vector");
  const KParams kp = kparams(ctx);
  if (precision == HF_FP64) {
    Ops<double> op{ctx->A, ctx->Bs, ctx->Cs, ctx->D, ctx->inv, ctx->Sinv};
    TRY(apply_J<double>(ctx, kp, op, (const double *)x, (double *)y));
  } else if (precision == HF_FP32_IR) {
    if (!ctx->have32) return fail(ctx, HF_ESTATE, "no FP32 matrix: run hf_solve in FP32-IR mode first");
    Ops<float> op{ctx->A32, ctx->Bs32, ctx->Cs32, ctx->D32, ctx->inv32, ctx->Sinv32};
    TRY(apply_J<float>(ctx, kp, op, (const float *)x, (float *)y));
  } else {
    return fail(ctx, HF_EINVAL, "precision");
  }
  return HF_OK;
}

extern "C" hf_status hf_get_profile(hf_ctx *ctx, hf_profile *out) {
  if (!ctx || !out) return HF_EINVAL;
  resolve_profile(ctx);
  *out = ctx->prof;
  return HF_OK;
}

extern "C" hf_status hf_reset_profile(hf_ctx *ctx) {
  if (!ctx) return HF_EINVAL;
  resolve_profile(ctx);
  std::memset(&ctx->prof, 0, sizeof(ctx->prof));
  return HF_OK;
}
