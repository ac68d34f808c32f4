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
constexpr int kChunkRows = 1024;  // rows of a reduction chunk of the batched Krylov kernels
constexpr int kMaxPressureBlock = 16384;  // pressure nodes per instance (dense pressure block)
constexpr int kGjPanel = 32;  // pivots per panel of the blocked Gauss-Jordan of large pressure blocks
constexpr int kDenseWideMin = 192;       // pressure blocks from this size are inverted grid-wide
// fixed device array of the allocation-free folded product (its S^-1 x_p
// staging vector): 512 KiB per GPU, i.e. 65,536 pressure unknowns per context
constexpr int64_t kNoAllocScratchBytes = 512 * 1024;
constexpr int64_t kNoAllocScratchElems = kNoAllocScratchBytes / 8;

// Rule tables of a context, in device memory owned by the context (each
// context has its own copy, so contexts of different element types can run
// concurrently on different streams).
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
// material and fluid-row scale of one instance
struct InstPar {
  double lam, G, sigma_c, delta_c, mu, dt, s_p, pad;
};

struct KParams {
  Sizes s;
  DevMesh m;
  const InstPar *ip;       // n_inst
  const int32_t *einst;    // ne: instance of each element
  const int32_t *pinst;    // n_p: instance of each pressure node
  const int32_t *poff;     // n_inst+1: first pressure node of each instance
  const int64_t *doff;     // n_inst+1: offset of each instance's dense pressure block
  const int32_t *aoff;     // n_inst+1: first active (fluid) face of each instance
  const RuleTables *rt;    // quadrature rules of the context (device)
  int n_inst;
  double b_stab;
  int freeze_p;  // 1: pressure held fixed (fluid rows become p-rows of the identity)
  int spmv_var = 0, prec_var = 0;  // lanes per element row: 0 wide, 1 half (tuning)
  const double *wmax = nullptr;    // nf*nq unloading history of the face points, or null (envelope only)
};

// device view of the batched Krylov state (see hf_kernels_krylov.hip)
struct KrylovDev {
  int n_inst = 0, n_chunks = 0;
  int ortho_var = 0;  // rows per thread of the Gram-Schmidt passes: 0 -> 4, 1 -> 8, 2 -> 2
  const int64_t *c_row0 = nullptr;
  const int32_t *c_len = nullptr, *c_inst = nullptr, *cptr = nullptr;
  int *solving = nullptr, *kconv = nullptr, *its = nullptr, *status = nullptr, *nbasis = nullptr;
  int *itmax = nullptr;  // per-instance cap on the iterations of the current solve
  double *rtol = nullptr;  // per-instance relative tolerance of the current solve
  double *bnorm = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr;
  double *L = nullptr;  // strictly lower Gram factor of the basis, packed by rows (single-pass MGS)
};

// rows a batched product works on: all (mode 0), the instances being solved
// (mode 1), or those still iterating in their GMRES cycle (mode 2)
struct RowSel {
  const int *solving = nullptr, *kconv = nullptr;
  int mode = 0;
};

// ---------------------------------------------------------------------------
// Two-level preconditioner: host structure (hf_coarse.cpp)
// ---------------------------------------------------------------------------
struct CoarseIn {  // the concatenated layout of a finalized context
  int dim = 0, order = 0, nn = 0, nq = 0, n_inst = 0, leaf_max = 64;
  int64_t ne = 0, nf = 0;
  const double *xyz = nullptr;
  const int32_t *elem = nullptr;
  const uint32_t *clamp = nullptr;
  const int32_t *face_em = nullptr, *face_ep = nullptr, *fperm_m = nullptr, *fperm_p = nullptr;
  const uint8_t *qp_state = nullptr, *beta = nullptr;
  const int64_t *blk_ptr = nullptr;
  const int32_t *blk_col = nullptr;
  const int32_t *nbr = nullptr;   // ne*(dim+1): neighbour across each local face, or -1
  const int64_t *eoff = nullptr;  // n_inst+1
};

struct CoarsePlan {
  int dim = 0, nv = 0, max_ap = 0;
  int32_t ncls = 0;
  std::vector<int32_t> cls_of;         // ne*nv: class of each vertex copy, or -1
  std::vector<double> xyz;             // ncls*dim
  std::vector<int32_t> cinst, coff;    // instance of each class; class offsets per instance
  std::vector<int32_t> rc_ptr, rc_list;  // copies (e*nv + v) of each class
  std::vector<int64_t> ap_ptr;         // ne+1: column classes of each element row of A P
  std::vector<int32_t> ap_cls;
  int64_t n_pairs = 0;                 // class pairs of A_c
  std::vector<int64_t> pair_cptr;      // npair+1: contributions (e, v | j << 8) of each pair
  std::vector<int32_t> pc_e, pc_vj;
  std::vector<int64_t> pair_dest;      // front offset of the pair's dim x dim block
  std::vector<int32_t> pair_ld;        // leading dimension of that front
  int n_nodes = 0, n_levels = 0;
  std::vector<int32_t> level_ptr, level_nodes, level_maxk, level_maxf;
  std::vector<int32_t> fk, ff;         // own and front size (DOFs) per node
  std::vector<int64_t> fo, uo;         // front storage offset; update-row offset
  std::vector<int64_t> fd_ptr;         // nodes+1: front positions (DOFs)
  std::vector<int32_t> fd_dof;         // global coarse DOF of each front position
  std::vector<int64_t> src0, src1;     // update rows of the children landing at each position
  std::vector<int64_t> ea_ptr;         // nodes+1: extend-add map of each node into its parent
  std::vector<int32_t> ea_map;         // (class level) parent front position of each struct class
  std::vector<int32_t> parent, child_slot;
  int64_t front_total = 0, upd_total = 0;
  double factor_flops = 0.0;
};
void build_coarse_plan(const CoarseIn &in, CoarsePlan &cp);

// device view of the plan (kernel argument, by value)
struct CoarseK {
  int dim = 0, nv = 0, nn = 0;
  int32_t ncls = 0;
  int64_t n_pairs = 0, front_total = 0;
  int nw[4] = {0, 0, 0, 0};  // P1 weights of the element nodes per local vertex
  int wn[4][4] = {};
  double ww[4][4] = {};
  const int32_t *cls_of = nullptr, *cinst = nullptr, *rc_ptr = nullptr, *rc_list = nullptr;
  const int64_t *ap_ptr = nullptr;
  const int32_t *ap_cls = nullptr;
  const int64_t *w_off = nullptr;  // per strip entry: offset of its W row
  const int64_t *pair_cptr = nullptr, *pair_dest = nullptr;
  const int32_t *pc_e = nullptr, *pc_vj = nullptr, *pair_ld = nullptr;
  const int32_t *level_ptr = nullptr, *level_nodes = nullptr, *children = nullptr;
  const int32_t *fk = nullptr, *ff = nullptr, *fd_dof = nullptr, *ea_map = nullptr;
  const int64_t *fo = nullptr, *uo = nullptr, *fd_ptr = nullptr, *src0 = nullptr, *src1 = nullptr, *ea_ptr = nullptr;
  const int64_t *cpo = nullptr;  // per node: offset of its Gauss-Jordan column-panel scratch
};
// per-level sizes the launchers need on the host
struct CoarseHostView {
  int n_levels = 0;
  std::vector<int32_t> level_ptr, level_maxk, level_maxf, level_maxf_minus_k;
  std::vector<int64_t> level_maxchild_upd;
};

hipError_t coarse_build_ap(const KParams &kp, const CoarseK &ck, const double *A, const int32_t *elist, int64_t n,
                           double *AP, hipStream_t st);
hipError_t coarse_build_w(const KParams &kp, const CoarseK &ck, const double *Cs, const double *inv,
                          const double *AP, double *W, hipStream_t st);
// fronts <- A_c entries, extend-add and Gauss-Jordan level by level;
// flag != 0 on a zero or non-finite pivot
hipError_t coarse_factor(const KParams &kp, const CoarseK &ck, const CoarseHostView &hv, const double *AP,
                         double *F, double *Cp, double *Dsc, int *flag, hipStream_t st);
hipError_t coarse_ptb(const KParams &kp, const CoarseK &ck, const double *Bs, int nrhs, double *R, hipStream_t st);
template <typename TF>
hipError_t coarse_solve_multi(const CoarseK &ck, const CoarseHostView &hv, const TF *F, const double *b,
                              int nrhs, double *upd, double *y, double *xs, hipStream_t st);
hipError_t coarse_s_correct(const KParams &kp, const CoarseK &ck, const double *W, const double *Z, int nrhs,
                            double *S, hipStream_t st);
// one coarse solve xs = A_c^-1 b; upd, y and the front vectors cv are scratch
template <typename T, typename TF>
hipError_t coarse_solve1(const CoarseK &ck, const CoarseHostView &hv, const TF *F, const T *b, T *upd, T *y, T *cv,
                         T *xs, hipStream_t st);
// q' = v_p - (Cf v_u + W z_c) per pressure row; w_p = v_p when wp != null
template <typename T>
hipError_t coarse_q(const KParams &kp, const CoarseK &ck, const T *Cf, const T *W, const T *vu, const T *vp,
                    const T *zc, T *qout, T *wp, hipStream_t st);
// rc = P^T v_u: P_e^T v_e per vertex copy into cpy (ne*nv*dim), then the
// sum over each class's copies
template <typename T>
hipError_t coarse_restrict2(const KParams &kp, const CoarseK &ck, const T *v, T *cpy, T *rc, hipStream_t st);
// z_c2 = z_c1 - Z_c z_p (Z_c: coarse rows x nrhs, the instance's pressure nodes)
template <typename T>
hipError_t coarse_zc2(const KParams &kp, const CoarseK &ck, const T *Z, int nrhs, const T *zc1, const T *zp, T *zc2,
                      hipStream_t st);
template <typename T>
hipError_t coarse_t(const KParams &kp, const CoarseK &ck, const T *AP, const T *Bs, const T *vu, const T *zp,
                    const T *zc, T *t, T *apz, hipStream_t st);
template <typename T>
hipError_t coarse_prolong_add(const KParams &kp, const CoarseK &ck, const T *zc, T *zu, hipStream_t st);
// y_p = S x_p with the dense per-instance pressure blocks S (one wave per row)
template <typename T>
hipError_t coarse_pgemv(const KParams &kp, const T *S, const T *x, T *y, hipStream_t st);
// nodes with a non-zero P1 weight for local vertex v and the weights
int vertex_node_weights(int dim, int order, int v, int *nodes, double *w);

}  // namespace hf

namespace hf {
// launchers (hf_kernels_*.hip)
hipError_t launch_geometry(const KParams &kp, hipStream_t st);
// R, the row panels, coupling strips and fluid rows; with elist only the row
// panels, residual rows and strips of the n_el listed elements (and every
// fluid row)
hipError_t launch_assemble(const KParams &kp, const double *u, const double *p,
                           const double *w_old, double *A, double *R, double *Bs,
                           double *Cs, double *D, const int32_t *elist, int64_t n_el,
                           hipStream_t st);
hipError_t launch_opening(const KParams &kp, const double *u, double *w, hipStream_t st);
hipError_t launch_wmax(const KParams &kp, const double *w, double *out, hipStream_t st);
// DG normal traction t.n at every face point (nf*nq)
hipError_t launch_face_traction(const KParams &kp, const double *u, double *tn, hipStream_t st);
// new interface states after the activation checks (nf*nq states, nf fluid flags)
hipError_t launch_activation(const KParams &kp, const double *tn, const double *w, uint8_t *qp_out,
                             uint8_t *beta_out, hipStream_t st);
hipError_t launch_fluid_volume(const KParams &kp, const double *u, double *partial, double *out,
                               hipStream_t st);
hipError_t launch_fill(double v, double *x, int64_t n, hipStream_t st);
// FP64 Gauss-Jordan inverses (and their FP32 copies when inv32 != null) of
// the diagonal blocks of the n elements in elist (all ne elements when elist
// is null, n = ne); flag[b] |= 1 on a zero or non-finite pivot in instance b
hipError_t launch_blockinv(const KParams &kp, const double *A, double *inv, float *inv32,
                           const int32_t *elist, int64_t n, int *flag, hipStream_t st);
// FP32 inverses of the 30 x 30 blocks of the n listed elements (every element
// when elist is null, n = ne) on the matrix cores; flag[b] |= 4 when
// a tile pivot fails in instance b (the caller falls back to launch_blockinv)
hipError_t launch_blockinv32_mfma(const KParams &kp, const double *A, float *inv32,
                                  const int32_t *elist, int64_t n, int *flag, hipStream_t st);
hipError_t launch_convert_panels(const KParams &kp, const int32_t *elist, int64_t n, const double *A,
                                 float *A32, hipStream_t st);
// folded preconditioned operator: Af = A_ef inv_f for the nblk blocks of the
// row panels in blist (every block when blist is null), Cf = C_e inv_e for
// every C strip entry (FP64 arithmetic)
template <typename TI, typename TO>
hipError_t launch_fold(const KParams &kp, const double *A, const double *Cs, const TI *inv, TO *Af, TO *Cf,
                       const int32_t *blist, int64_t nblk, hipStream_t st);
// flag[b] |= 2 on a zero or non-finite pivot in the pressure block of instance b;
// the inverses of blocks with n_wide <= n (n_wide > 0) are left to
// launch_dense_inv_wide
hipError_t launch_schur(const KParams &kp, const double *inv, const double *Bs,
                        const double *Cs, const double *D, double *Z, double *T, double *S,
                        double *Sinv, float *Sinv32, int *flag, int n_wide, hipStream_t st);
// S = D - C M_A^-1 B only (no inversion)
hipError_t launch_schur_form(const KParams &kp, const double *inv, const double *Bs, const double *Cs,
                             const double *D, double *T, double *S, hipStream_t st);
// in-place inversion of the pressure blocks of S into Sinv / Sinv32 (the
// blocks with n_wide <= n are left to launch_dense_inv_wide)
hipError_t launch_schur_invert(const KParams &kp, double *S, double *Sinv, float *Sinv32, int *flag, int n_wide,
                               hipStream_t st);
// inverse of one n x n block W (row-major, in place) into out / out32 by
// Gauss-Jordan with partial pivoting blocked over panels of kGjPanel pivots
// (n <= kMaxPressureBlock); scratch colk ((kGjPanel + 1) kMaxPressureBlock
// doubles), perm (2 kMaxPressureBlock ints), piv (1); flag |= 2 on a zero or
// non-finite pivot
hipError_t launch_dense_inv_wide(double *W, double *out, float *out32, int n, int *flag, double *colk, int *perm,
                                 double *piv, hipStream_t st);
hipError_t launch_convert(const double *in, float *out, int64_t n, hipStream_t st);
// y[i] = max(y[i], x[i]), i < n
hipError_t launch_max_into(const double *x, double *y, int64_t n, hipStream_t st);
// staggered iteration, fluid half: row node[b] of instance b's pressure block
// W (a copy of D) becomes the identity row, R_p[node] = p[node] - value[b]
hipError_t launch_stag_dirichlet(const KParams &kp, const int32_t *node, const double *value,
                                 const double *p, double *W, double *Rp, hipStream_t st);
// dp = -Winv R_p per instance (Winv: the inverted pressure blocks)
hipError_t launch_stag_dp(const KParams &kp, const double *Winv, const double *Rp, double *dp,
                          hipStream_t st);
// y = J x (rows outside sel are left untouched)
template <typename T>
hipError_t launch_spmv(const KParams &kp, const T *A, const T *Bs, const T *Cs, const T *D,
                       const T *x, T *y, const RowSel &sel, hipStream_t st);
// y = J M^-1 x with the folded blocks: t_p = S^-1 x_p (into tp, n_p values),
// y_u = Af x_u + B t_p, y_p = Cf x_u + D t_p (rows outside sel untouched)
template <typename T>
hipError_t launch_spmv_folded(const KParams &kp, const T *Af, const T *Bs, const T *Cf, const T *D,
                              const T *Sinv, const T *x, T *y, T *tp, const RowSel &sel, hipStream_t st);
// device address of the fixed scratch array on `device`, which must be the
// current device; resolved once per device and kept
hipError_t noalloc_scratch(int device, void **ptr);
// element rows of the folded product with the pressure staging given:
// y_u = Af x_u + B tp + add (add nullable)
template <typename T>
hipError_t launch_spmv_folded_rows(const KParams &kp, const T *Af, const T *Bs, const T *x, const T *tp,
                                   const T *add, T *y, hipStream_t st);
// y_e = sum_f A_ef x_f for the element rows with skip[e] == 0 (no strips,
// no pressure rows; the other rows are left untouched)
hipError_t launch_spmv_rows(const KParams &kp, const double *A, const double *x, double *y,
                            const uint8_t *skip, hipStream_t st);
// r = b - J x in FP64 with compensated (double-double) accumulation (rows
// outside sel are left untouched)
hipError_t launch_resid(const KParams &kp, const double *A, const double *Bs, const double *Cs, const double *D,
                        const double *x, const double *b, double *r, const RowSel &sel, hipStream_t st);
// z = M^-1 r, block-Jacobi (rows outside sel are left untouched)
template <typename T>
hipError_t launch_precond(const KParams &kp, const T *inv, const T *Sinv, const T *r, T *z,
                          const RowSel &sel, hipStream_t st);
hipError_t launch_axpby(double a, const double *x, double b, double *y, int64_t n,
                        hipStream_t st);
// out[b] = ||x_b||^2 of every instance
hipError_t launch_seg_norms(const KrylovDev &kd, const double *x, double *partial, double *out,
                            hipStream_t st);
// out[4b + 0..3] = ||r_u||^2, ||b_u||^2, ||r_p||^2, ||b_p||^2 of instance b
// (displacement and pressure rows of two context vectors)
hipError_t launch_seg_norms_up(const KrylovDev &kd, const double *r, const double *b, int64_t n_u,
                               double *partial, double *out, hipStream_t st);
// x += dx on instances with upd[b] != 0 (p clamped to the cut-off when on);
// out[4b + 0..3] = ||du||^2, ||u||^2, ||dp||^2, ||p||^2 of instance b
hipError_t launch_snewton_update(const KrylovDev &kd, const double *dx, double *x, int64_t n_u,
                                 const int *upd, int cutoff_on, double cutoff, double *partial,
                                 double *out, hipStream_t st);

// batched Krylov (hf_kernels_krylov.hip)
template <typename T>
hipError_t ks_proj(const KrylovDev &kd, const T *V, int64_t ldv, int k, const T *w,
                   const int *gate, double *partial, double *out, hipStream_t st);
template <typename T>
hipError_t ks_update(const KrylovDev &kd, const T *V, int64_t ldv, int k, const double *h,
                     int hstride, T *w, const int *gate, double *partial, double *out,
                     hipStream_t st);
template <typename T>
hipError_t ks_scale(const KrylovDev &kd, const T *w, const double *scale, T *v, hipStream_t st);
template <typename T>
hipError_t ks_combine(const KrylovDev &kd, const T *V, int64_t ldv, const double *y, int ystride,
                      T *out, hipStream_t st);
template <typename TX, typename TZ>
hipError_t ks_axpy(const KrylovDev &kd, const double *coef, const TZ *z, TX *x, hipStream_t st);
template <typename T>
hipError_t ks_sub(const KrylovDev &kd, const T *b, const T *jx, T *r, hipStream_t st);
template <typename TY, typename TX>
hipError_t ks_cast(const KrylovDev &kd, const TX *x, const double *coef, TY *y, hipStream_t st);
// y = x on the rows of iterating instances
hipError_t ks_copy(const KrylovDev &kd, const double *x, double *y, hipStream_t st);
template <typename T>
hipError_t ks_zero(const KrylovDev &kd, T *x, int only_solving, hipStream_t st);
// flag[b] = 1 when instance b takes a second Gram-Schmidt pass: policy 0 when
// ||w1||^2 < ||w||^2 / 2 (n1, n0), 1 always, 2 never
hipError_t ks_reorth_flag(const KrylovDev &kd, const double *n0, int n0s, const double *n1, int policy,
                          int *flag, hipStream_t st);
// ||w||^2 from n2[b] (second pass) or n1[b], or, with pnorm, summed from the
// last update's chunk partials (where n1 is null or the second pass ran)
hipError_t ks_arnoldi(const KrylovDev &kd, int j, int m, const double *s1, int s1s, const double *s2,
                      int s2s, const int *reorth, const double *n1, const double *n2, const double *pnorm,
                      double *scale, hipStream_t st);
// one-reduce projection for the single-pass modified Gram-Schmidt: out (per
// instance, stride 2k-1) = V_{0..k-1}^T w, then V_{0..k-2}^T v_{k-1}
template <typename T>
hipError_t ks_proj2(const KrylovDev &kd, const T *V, int64_t ldv, int k, const T *w, double *partial,
                    double *out, hipStream_t st);
// h (stride hstride) = (I + L)^-1 s with row j of L taken from sv and stored
// in Lmat ((m+1) x (m+1) per instance)
hipError_t ks_icwy(const KrylovDev &kd, int j, int m, const double *sv, double *Lmat, double *h,
                   int hstride, hipStream_t st);
// out[b] = ||x_b||^2 for every instance (no gating)
template <typename T>
hipError_t ks_norms(const KrylovDev &kd, const T *x, double *partial, double *out, hipStream_t st);
// start of a solve: bnorm = sqrt(n2), kconv = -1, its = 0, status = 0
hipError_t ks_begin(const KrylovDev &kd, const double *n2, hipStream_t st);
hipError_t ks_count_active(const KrylovDev &kd, int *count, hipStream_t st);
hipError_t ks_solve_y(const KrylovDev &kd, int m, double *y, double *est, hipStream_t st);
hipError_t ks_cycle_start(const KrylovDev &kd, int m, const double *beta2, double *scale,
                          hipStream_t st);
}  // namespace hf
