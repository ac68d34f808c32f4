// Internal declarations of the hydraulic-fracture Newton-step library:
// host layout, device buffers, kernel parameter blocks and launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hf.h"

namespace hf {

// ---------------------------------------------------------------------------
// Quadrature rules and reference data computed on the host (hf_rules.cpp).
// ---------------------------------------------------------------------------
struct Rule {
  int dim = 0;                 // dimension of the simplex
  std::vector<double> pts;     // nq * dim reference coordinates
  std::vector<double> w;       // nq weights
  int nq() const { return (int)w.size(); }
};
// Conical-product Gauss rule with n points per direction on the reference
// simplex of dimension dim (weights sum to its measure).
Rule simplex_rule(int dim, int n);

constexpr int kMaxNq = 9;      // face points of 3D P2 (3 x 3)
constexpr int kMaxKrylov = 257;  // basis vectors (restart length + 1)
constexpr int kMaxNqv = 8;     // volume points of 3D P2 (2 x 2 x 2)

// Rule tables, in the device constant bank (set per context before launch).
struct RuleTables {
  double fq_mu[kMaxNq][3];     // face barycentrics over the sorted face vertices
  double fq_w[kMaxNq];         // face weights, sum 1
  double vq_lam[kMaxNqv][4];   // volume barycentrics
  double vq_w[kMaxNqv];        // volume weights, sum = reference measure
  int nqf, nqv;
};

// ---------------------------------------------------------------------------
// Device buffers of one instance
// ---------------------------------------------------------------------------
template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
};

struct DevMesh {
  // geometry
  double *xyz = nullptr;        // n_vert*dim
  int32_t *elem_vert = nullptr; // ne*(dim+1)
  double *gl = nullptr;         // ne*(dim+1)*dim   gradients of barycentrics
  double *detabs = nullptr;     // ne               |det J|
  int32_t *nbr = nullptr;       // ne*(dim+1)       neighbour across local face or -1
  int32_t *fid = nullptr;       // ne*(dim+1)       interior face id or -1
  int32_t *blk_of = nullptr;    // ne*(dim+1)       block index of the off-diagonal block
  uint32_t *clamp = nullptr;    // ne               bit r = DOF row r clamped
  int64_t *blk_ptr = nullptr;   // ne+1             first block of each element row
  int32_t *blk_col = nullptr;   // n_blocks
  // faces
  int32_t *face_vert = nullptr; // nf*dim
  int32_t *face_em = nullptr, *face_ep = nullptr;
  int32_t *fperm_m = nullptr, *fperm_p = nullptr;  // nf*dim local vertex of face vertex k
  int32_t *face_lfm = nullptr;  // nf local face index in e- (its opposite vertex)
  double *normal = nullptr;     // nf*dim
  double *area = nullptr;       // nf
  double *hf = nullptr;         // nf
  double *ginv = nullptr;       // nf*(dim-1)^2  inverse face metric
  uint8_t *qp_state = nullptr;  // nf*nq
  uint8_t *beta = nullptr;      // nf
  int32_t *slot = nullptr;      // nf  active-face slot or -1
  // pressure skeleton
  int32_t *act_face = nullptr;  // n_act
  int32_t *face_pn = nullptr;   // n_act*nnf
  int32_t *fs_idx = nullptr;    // ne*(dim+1)*nnf strip entry of (element, face, node) or -1
  int64_t *sp_ptr = nullptr;    // ne+1 strip entries per element
  int32_t *sp_pnode = nullptr;  // n_strip
  int32_t *sp_elem = nullptr;   // n_strip
  int32_t *pc_ptr = nullptr;    // n_p+1 strip entries per pressure node
  int32_t *pc_ent = nullptr;    // n_strip
  int32_t *pf_ptr = nullptr;    // n_p+1 (active face, local node) per pressure node
  int32_t *pf_fa = nullptr, *pf_k = nullptr;
  int32_t *src_node = nullptr;  // n_src
  double *src_q0 = nullptr;
  int32_t *strip_elems = nullptr;  // n_se elements owning strips
  int32_t *sp_se = nullptr;     // n_strip strip-element index of each entry
  int64_t *t_ptr = nullptr;     // n_se+1 offsets of the Schur staging blocks
  int64_t *ident_ptr = nullptr; // ne+1 identity block pattern (block-diagonal apply)
  int32_t *ident_col = nullptr; // ne
};

struct Sizes {
  int dim = 0, order = 0, nn = 0, bu = 0, nnf = 0, nqf = 0, nqv = 0;
  int64_t n_vert = 0, ne = 0, nf = 0, n_u = 0, n_p = 0, n_act = 0, n_blocks = 0;
  int64_t n_strip = 0, n_se = 0, n_t = 0, n_src = 0;
  int64_t N() const { return n_u + n_p; }
};

// ---------------------------------------------------------------------------
// Kernel parameter block (passed by value)
// ---------------------------------------------------------------------------
struct KParams {
  Sizes s;
  DevMesh m;
  double lam, G, sigma_c, delta_c, mu, dt, b_stab, s_p;
  int freeze_p;  // 1: pressure held fixed (fluid rows become p-rows of the identity)
};

// ---------------------------------------------------------------------------
// Host-side layout built by hf_upload_mesh / hf_finalize
// ---------------------------------------------------------------------------
struct HostLayout {
  std::vector<double> xyz;
  std::vector<int32_t> elem;            // ne*(dim+1)
  std::vector<uint8_t> dirichlet;       // n_vert
  std::vector<int32_t> face_vert;       // nf*dim (sorted)
  std::vector<int32_t> face_em, face_ep, fperm_m, fperm_p, face_lfm;
  std::vector<int32_t> nbr, fid;        // ne*(dim+1)
  std::vector<uint32_t> clamp;          // ne
  std::vector<uint8_t> qp_state, beta;
  std::vector<int64_t> src_vert;
  std::vector<double> src_q0;
  // finalize
  std::vector<int64_t> pkeys;           // n_p*2
  std::vector<int32_t> act_face, face_pn, slot;
  double bbox_L = 1.0;
};

struct Material {
  double E = 1, nu = 0.25, sigma_c = 1e-3, G_c = 1e-4, mu = 1e-3, dt = 1;
  bool set = false;
};

}  // namespace hf

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
namespace hf {
template <typename T>
struct KrylovWs {
  T *V = nullptr;   // (m+1) x N basis, column i at V + i*N
  T *w = nullptr, *z = nullptr, *r = nullptr, *t = nullptr, *b = nullptr, *x = nullptr;
  int m = 0;
  int64_t n = 0;
};
}  // namespace hf

struct hf_ctx {
  hf_options opt{};
  std::string err;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int stage = 0;  // 0 created, 1 mesh, 2 finalized, 3 state set, 4 assembled, 5 solved
  hf::Sizes s;
  hf::HostLayout h;
  hf::Material mat;
  hf::DevMesh m;
  hf::RuleTables rules{};
  double s_p = 1.0;
  int freeze_p = 0;
  int64_t n_reorth = 0;         // Gram-Schmidt re-orthogonalisations taken (diagnostic)
  std::vector<void *> allocs;   // every device allocation, released by hf_destroy
  // state: xs = [u; p]
  double *xs = nullptr, *xs_save = nullptr, *xs_start = nullptr, *w_old = nullptr, *w_tmp = nullptr;
  // assembled system
  double *R = nullptr;          // N residual
  double *A = nullptr;          // n_blocks*bu*bu (column-major blocks, row panels)
  double *Bs = nullptr, *Cs = nullptr;      // n_strip*bu coupling strips
  double *D = nullptr, *S = nullptr, *Sinv = nullptr;   // n_p*n_p dense
  double *T = nullptr;          // Schur staging
  double *inv = nullptr;        // ne*bu*bu block inverses (column-major)
  float *A32 = nullptr, *Bs32 = nullptr, *Cs32 = nullptr, *D32 = nullptr, *Sinv32 = nullptr;
  float *inv32 = nullptr;
  bool have32 = false;          // FP32 copies current
  int *flag = nullptr;          // device error flags
  // FP64 work vectors
  double *dx = nullptr, *rhs = nullptr, *r64 = nullptr, *t64 = nullptr;
  hf::KrylovWs<double> k64;
  hf::KrylovWs<float> k32;
  double *partial = nullptr;    // reduction partials
  double *red = nullptr;        // reduction results (device)
  double *red_h = nullptr;      // pinned host copy
  // profile: events recorded around kernel classes without host waits,
  // resolved into totals by hf_get_profile
  std::vector<hipEvent_t> evpool;
  size_t ev_used = 0;
  std::vector<std::array<int64_t, 3>> ev_pending;  // (class, start event, end event)
  hf_profile prof{};
};

namespace hf {
// launchers (hf_kernels_*.hip)
hipError_t launch_geometry(const KParams &kp, hipStream_t st);
hipError_t launch_assemble(const KParams &kp, const double *u, const double *p,
                           const double *w_old, double *A, double *R, double *Bs,
                           double *Cs, double *D, hipStream_t st);
hipError_t launch_opening(const KParams &kp, const double *u, double *w, hipStream_t st);
hipError_t launch_wmax(const KParams &kp, const double *w, double *out, hipStream_t st);
hipError_t launch_fluid_volume(const KParams &kp, const double *u, double *partial, double *out,
                               hipStream_t st);
hipError_t launch_fill(double v, double *x, int64_t n, hipStream_t st);
hipError_t launch_blockinv(const KParams &kp, const double *A, double *inv, float *inv32,
                           int *flag, hipStream_t st);
hipError_t launch_schur(const KParams &kp, const double *inv, const double *Bs,
                        const double *Cs, const double *D, double *Z, double *T, double *S,
                        double *Sinv, float *Sinv32, int *flag, hipStream_t st);
hipError_t launch_convert(const double *in, float *out, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_spmv(const KParams &kp, const T *A, const T *Bs, const T *Cs, const T *D,
                       const T *x, T *y, hipStream_t st);
template <typename T>
hipError_t launch_precond(const KParams &kp, const T *inv, const T *Sinv, const T *r, T *z,
                          hipStream_t st);
// Krylov BLAS (deterministic two-stage reductions)
int reduce_blocks(int64_t n);
int ortho_blocks(int64_t n);  // blocks of the Gram-Schmidt passes (partials per output)
template <typename T>
hipError_t launch_mdot(const T *V, int64_t ldv, int k, const T *w, int64_t n, double *partial,
                       double *out, hipStream_t st);
template <typename T>
hipError_t launch_update_mdot(const T *V, int64_t ldv, int k, const double *h, T *w, int64_t n,
                              double *partial, double *out, hipStream_t st);
template <typename T>
hipError_t launch_update_norm(const T *V, int64_t ldv, int k, const double *h, T *w, int64_t n,
                              double *partial, double *out, hipStream_t st);
// Gram-Schmidt passes: out[0..k) = V^T w, out[k] = ||w||^2; and w -= V h, out[0] = ||w||^2
template <typename T>
hipError_t launch_proj(const T *V, int64_t ldv, int k, const T *w, int64_t n, double *partial,
                       double *out, hipStream_t st);
template <typename T>
hipError_t launch_orth_update(const T *V, int64_t ldv, int k, const double *h, T *w, int64_t n,
                              double *partial, double *out, hipStream_t st);
template <typename T>
hipError_t launch_scale_copy(const T *w, double inv_norm, T *v, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_combine(const T *V, int64_t ldv, int k, const double *y, T *out, int64_t n,
                          hipStream_t st);
hipError_t launch_axpby(double a, const double *x, double b, double *y, int64_t n,
                        hipStream_t st);
hipError_t launch_cast_axpy(double a, const float *x, double *y, int64_t n, hipStream_t st);
hipError_t launch_cast_scale(const double *x, double a, float *y, int64_t n, hipStream_t st);
hipError_t launch_sub(const double *b, const double *Jx, double *r, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_sub_t(const T *b, const T *Jx, T *r, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_axpy_t(double a, const T *x, T *y, int64_t n, hipStream_t st);
hipError_t launch_newton_update(const double *dx, double *u, int64_t n_u, double *p,
                                int64_t n_p, int cutoff_on, double cutoff, double *partial,
                                double *out, hipStream_t st);
hipError_t launch_norm2(const double *x, int64_t n, double *partial, double *out,
                        hipStream_t st);
hipError_t launch_set_rules(const RuleTables &rt, hipStream_t st);
}  // namespace hf
