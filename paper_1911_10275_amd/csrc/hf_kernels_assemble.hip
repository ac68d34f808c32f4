// Assembly kernels for gfx950: geometry, the element-centric residual and
// Jacobian rows of the displacement equations, the fluid rows, and the
// opening at face points.
//
// Element-centric assembly: every element (one workgroup) computes its own
// row of blocks -- the diagonal block (bulk term plus the self part of each of
// its interface elements) and one off-diagonal block per interior face -- so
// every block is written exactly once, with a fixed summation order, no
// atomics and no staging.  Each interface integral is therefore evaluated by
// both of its elements, each for its own test functions.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "hf_internal.h"

namespace hf {

// Grid of a persistent kernel: the workgroups of one kernel that the device
// holds at once (its occupancy per CU times the CU count), capped at the
// number of work items.  Queried once per device and kernel, then kept.
class ResidentGrid {
 public:
  hipError_t size(const void *kernel, int threads, int64_t n_items, unsigned *grid) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu_);
    if ((int)cap_.size() <= dev) cap_.resize(dev + 1, 0);
    if (cap_[dev] <= 0) {
      int occ = 0, ncu = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0);
      if (e != hipSuccess) return e;
      e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      cap_[dev] = std::max(occ, 1) * std::max(ncu, 1);
    }
    *grid = (unsigned)std::min<int64_t>(n_items, cap_[dev]);
    return hipSuccess;
  }

 private:
  std::mutex mu_;
  std::vector<int64_t> cap_;
};

// ---------------------------------------------------------------------------
// Lagrange P1/P2 on simplices in barycentric coordinates
// node order: vertices, then edges (01),(12),(20),(03),(13),(23)
// ---------------------------------------------------------------------------
template <int D, int K>
struct Lag {
  static constexpr int NN = (K == 1) ? D + 1 : (D + 1) * (D + 2) / 2;
  __device__ static constexpr int ea(int k) {
    return k < 3 ? (D == 1 ? 0 : k) : k - 3;
  }
  __device__ static constexpr int eb(int k) {
    return D == 1 ? 1 : (k < 3 ? (k + 1) % 3 : 3);
  }
  __device__ static void phi(const double *lam, double *out) {
    if (K == 1) {
#pragma unroll
      for (int a = 0; a <= D; ++a) out[a] = lam[a];
    } else {
#pragma unroll
      for (int a = 0; a <= D; ++a) out[a] = lam[a] * (2.0 * lam[a] - 1.0);
#pragma unroll
      for (int k = 0; k < NN - D - 1; ++k) out[D + 1 + k] = 4.0 * lam[ea(k)] * lam[eb(k)];
    }
  }
  // one basis function and its barycentric derivatives
  __device__ static double phi_one(int a, const double *lam) {
    if (K == 1) return lam[a];
    if (a <= D) return lam[a] * (2.0 * lam[a] - 1.0);
    const int k = a - D - 1;
    return 4.0 * lam[ea(k)] * lam[eb(k)];
  }
  __device__ static void dphi_one(int a, const double *lam, double *out) {
    for (int k = 0; k <= D; ++k) out[k] = 0.0;
    if (K == 1) {
      out[a] = 1.0;
    } else if (a <= D) {
      out[a] = 4.0 * lam[a] - 1.0;
    } else {
      const int k = a - D - 1;
      out[ea(k)] = 4.0 * lam[eb(k)];
      out[eb(k)] = 4.0 * lam[ea(k)];
    }
  }
  // Every P1/P2 node function in one product form, phi_a = c1 lam_i lam_j +
  // c2 lam_i (vertex of P2: i = j = a, c1 = 2, c2 = -1; edge (i, j): c1 = 4,
  // c2 = 0; P1: i = j = a, c1 = 0, c2 = 1), so that its gradient is
  // c1 (lam_j grad lam_i + lam_i grad lam_j) + c2 grad lam_i without branches.
  __device__ static void node_form(int a, int &i, int &j, double &c1, double &c2) {
    if (K == 1) {
      i = a;
      j = a;
      c1 = 0.0;
      c2 = 1.0;
    } else {
      const bool v = a <= D;
      const int k = v ? 0 : a - D - 1;
      i = v ? a : ea(k);
      j = v ? a : eb(k);
      c1 = v ? 2.0 : 4.0;
      c2 = v ? -1.0 : 0.0;
    }
  }
  // d phi_a / d lam_k
  __device__ static void dphi(const double *lam, double out[][D + 1]) {
#pragma unroll
    for (int a = 0; a < NN; ++a)
#pragma unroll
      for (int k = 0; k <= D; ++k) out[a][k] = 0.0;
    if (K == 1) {
#pragma unroll
      for (int a = 0; a <= D; ++a) out[a][a] = 1.0;
    } else {
#pragma unroll
      for (int a = 0; a <= D; ++a) out[a][a] = 4.0 * lam[a] - 1.0;
#pragma unroll
      for (int k = 0; k < NN - D - 1; ++k) {
        out[D + 1 + k][ea(k)] = 4.0 * lam[eb(k)];
        out[D + 1 + k][eb(k)] = 4.0 * lam[ea(k)];
      }
    }
  }
};

template <int DIM, int ORDER>
struct Cfg {
  static constexpr int NN = Lag<DIM, ORDER>::NN;
  static constexpr int BU = NN * DIM;
  static constexpr int NF = DIM + 1;
  static constexpr int NQF = (DIM == 2) ? ORDER + 1 : (ORDER + 1) * (ORDER + 1);
  static constexpr int NQV = (DIM == 2) ? ORDER * ORDER : ORDER * ORDER * ORDER;
  static constexpr int NNF = Lag<DIM - 1, ORDER>::NN;
};

// ---------------------------------------------------------------------------
// Geometry: gradients of barycentrics, |det J|; face normal, area, h, metric
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void k_geom_elem(KParams kp) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= kp.s.ne) return;
  const int32_t *ev = kp.m.elem_vert + e * (DIM + 1);
  double X0[DIM], J[DIM][DIM];
  for (int c = 0; c < DIM; ++c) X0[c] = kp.m.xyz[(int64_t)ev[0] * DIM + c];
  for (int k = 0; k < DIM; ++k)
    for (int c = 0; c < DIM; ++c) J[c][k] = kp.m.xyz[(int64_t)ev[k + 1] * DIM + c] - X0[c];
  double Ji[DIM][DIM], det;
  if constexpr (DIM == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
  } else {
    // inverse = adjugate / det, adjugate = cofactor^T
    double cof[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        int r1 = (r + 1) % 3, r2 = (r + 2) % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        cof[r][c] = J[r1][c1] * J[r2][c2] - J[r1][c2] * J[r2][c1];
      }
    det = J[0][0] * cof[0][0] + J[0][1] * cof[0][1] + J[0][2] * cof[0][2];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) Ji[r][c] = cof[c][r] / det;
  }
  double *gl = kp.m.gl + e * (DIM + 1) * DIM;
  for (int x = 0; x < DIM; ++x) {
    double s = 0.0;
    for (int k = 0; k < DIM; ++k) {
      gl[(k + 1) * DIM + x] = Ji[k][x];
      s += Ji[k][x];
    }
    gl[x] = -s;
  }
  kp.m.detabs[e] = fabs(det);
}

template <int DIM>
__global__ void k_geom_face(KParams kp) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= kp.s.nf) return;
  const int32_t *fv = kp.m.face_vert + f * DIM;
  double V[DIM][DIM];
  for (int k = 0; k < DIM; ++k)
    for (int c = 0; c < DIM; ++c) V[k][c] = kp.m.xyz[(int64_t)fv[k] * DIM + c];
  double n[DIM], area;
  double t1[DIM];
  for (int c = 0; c < DIM; ++c) t1[c] = V[1][c] - V[0][c];
  if constexpr (DIM == 2) {
    n[0] = t1[1];
    n[1] = -t1[0];
    area = sqrt(n[0] * n[0] + n[1] * n[1]);
    kp.m.ginv[f] = 1.0 / (t1[0] * t1[0] + t1[1] * t1[1]);
  } else {
    double t2[3];
    for (int c = 0; c < 3; ++c) t2[c] = V[2][c] - V[0][c];
    n[0] = t1[1] * t2[2] - t1[2] * t2[1];
    n[1] = t1[2] * t2[0] - t1[0] * t2[2];
    n[2] = t1[0] * t2[1] - t1[1] * t2[0];
    double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    area = 0.5 * nn;
    double g11 = t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2];
    double g22 = t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2];
    double g12 = t1[0] * t2[0] + t1[1] * t2[1] + t1[2] * t2[2];
    double dg = g11 * g22 - g12 * g12;
    double *gi = kp.m.ginv + f * 4;
    gi[0] = g22 / dg;
    gi[1] = -g12 / dg;
    gi[2] = -g12 / dg;
    gi[3] = g11 / dg;
  }
  // orient outward of the minus element: away from its vertex opposite the face
  int32_t em = kp.m.face_em[f], ep = kp.m.face_ep[f];
  int32_t vopp = kp.m.elem_vert[(int64_t)em * (DIM + 1) + kp.m.face_lfm[f]];
  double dotv = 0.0, nrm = 0.0;
  for (int c = 0; c < DIM; ++c) {
    dotv += n[c] * (kp.m.xyz[(int64_t)vopp * DIM + c] - V[0][c]);
    nrm += n[c] * n[c];
  }
  nrm = sqrt(nrm);
  double sg = dotv > 0.0 ? -1.0 : 1.0;
  for (int c = 0; c < DIM; ++c) kp.m.normal[f * DIM + c] = sg * n[c] / nrm;
  kp.m.area[f] = area;
  const double fact = (DIM == 2) ? 2.0 : 6.0;
  double vm = kp.m.detabs[em] / fact, vp = kp.m.detabs[ep] / fact;
  kp.m.hf[f] = fmin(vm, vp) / area;
}

hipError_t launch_geometry(const KParams &kp, hipStream_t st) {
  const int nt = 128;
  int ge = (int)((kp.s.ne + nt - 1) / nt), gf = (int)((kp.s.nf + nt - 1) / nt);
  if (kp.s.dim == 2) {
    if (ge) hipLaunchKernelGGL(k_geom_elem<2>, dim3(ge), dim3(nt), 0, st, kp);
    if (gf) hipLaunchKernelGGL(k_geom_face<2>, dim3(gf), dim3(nt), 0, st, kp);
  } else {
    if (ge) hipLaunchKernelGGL(k_geom_elem<3>, dim3(ge), dim3(nt), 0, st, kp);
    if (gf) hipLaunchKernelGGL(k_geom_face<3>, dim3(gf), dim3(nt), 0, st, kp);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Interface law (normal cohesive traction) and cubic-law conductivity
// ---------------------------------------------------------------------------
// wm: the point's unloading history (0: none).  A cohesive point that has
// opened to wm > 0 and stands below it unloads on the secant to the origin,
// T = (T_env(wm) / wm) w, and meets plain contact k_c w once closed.
__device__ inline void traction_law(int state, double w, double sigma_c, double delta_c,
                                    double kc, double wm, double &T, double &dT) {
  T = 0.0;
  dT = 0.0;
  if (state == 1) {
    if (wm > 0.0 && w < wm) {
      if (w < 0.0) {
        T = kc * w;
        dT = kc;
      } else {
        const double ks = (wm <= delta_c ? sigma_c * (1.0 - wm / delta_c) : 0.0) / wm;
        T = ks * w;
        dT = ks;
      }
    } else if (w < 0.0) {
      T = sigma_c + kc * w;
      dT = kc;
    } else if (w <= delta_c) {
      T = sigma_c * (1.0 - w / delta_c);
      dT = -sigma_c / delta_c;
    }
  } else if (state == 2) {
    if (w < 0.0) {
      T = kc * w;
      dT = kc;
    }
  }
}

// ---------------------------------------------------------------------------
// Element-centric assembly of the displacement rows.
//
// Interface blocks.  With c_qa = W_q s_e phi^e_a(x_q) (s_e = -1 on the minus
// side, +1 on the plus side), the block of test node a / trial node b of side
// t is
//   B[a i][b j] = lam/2 n_i M1[a][b][j] + G/2 n_j M1[a][b][i] + G/2 d_ij M2[a][b]
//               + (b/h) s_t Chat_ij M3[a][b] + s_t n_i n_j M4[a][b]
// with the moment matrices over the face points
//   M1[a][b][x] = sum_q c_qa (1-alpha_q) dphi^t_b/dx_x,  M2 = sum_q c_qa (1-alpha_q) grad phi^t_b . n,
//   M3[a][b]    = sum_q c_qa (1-alpha_q) phi^t_b,         M4 = sum_q c_qa alpha_q T'(w_q) phi^t_b,
// which is the derivative of the interface traction
//   tau = (1-alpha)(<sigma(u)> n + (b/h) Chat [[u]]) + alpha T(w) n - beta p n
// tested with s_e phi^e_a e_i.  Bulk block: K[a i][b j] = lam P[a][b][i][j]
// + G d_ij tr P[a][b] + G P[a][b][j][i], P[a][b][x][y] = sum_q w_q |det J|
// dphi_a/dx_x dphi_b/dx_y.
// ---------------------------------------------------------------------------
template <int DIM, int ORDER, int NT>
__device__ __forceinline__ void assemble_element(const KParams &kp, const RuleTables &rt,
                                                 const int64_t e,
                                                 const double *__restrict__ u,
                                                 const double *__restrict__ p,
                                                 const double *__restrict__ w_old,
                                                 double *__restrict__ A, double *__restrict__ R,
                                                 double *__restrict__ Bs,
                                                 double *__restrict__ Cs) {
  using C = Cfg<DIM, ORDER>;
  constexpr int NN = C::NN, BU = C::BU, NF = C::NF, NQF = C::NQF, NQV = C::NQV, NNF = C::NNF;
  constexpr int NQ = NQF > NQV ? NQF : NQV;
  constexpr int NG = (DIM - 1) * (DIM - 1);
  // An empty asm that claims to change the thread index keeps the compiler from
  // hoisting every phase's per-thread LDS addresses out of the element and face
  // loops (kept live across all phases, they would double the register count).
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const InstPar P = kp.ip[kp.einst[e]];
  const double lam = P.lam, G = P.G;

  __shared__ double s_gl[NF][DIM];
  __shared__ double s_ue[BU];
  __shared__ double s_diag[BU * BU];
  __shared__ double s_phE[NQ][NN], s_gphE[NQ][NN][DIM];
  __shared__ double s_phN[NQF][NN], s_gphN[NQF][NN][DIM];
  __shared__ double s_gu[NQV][DIM][DIM];      // displacement gradient at the volume points
  __shared__ double s_gj[NQF][DIM][DIM + 1];  // averaged gradient and jump at the face points
  __shared__ double s_gnE[NQF][NN], s_gnN[NQF][NN];  // grad phi . n at the face points
  __shared__ double s_tau[NQF][DIM], s_W[NQF];
  __shared__ double s_c1[NQF], s_c4[NQF];  // W_q s_e (1 - alpha_q), W_q s_e alpha_q T'(w_q)
  __shared__ double s_eta[NQF][NNF], s_fc[NQF][NNF];
  __shared__ double s_R[BU];
  // every interface element of this element, read once up front
  __shared__ int32_t s_f[NF], s_nb[NF], s_slot[NF], s_beta[NF], s_minus[NF];
  __shared__ int32_t s_pe[NF][DIM], s_pn[NF][DIM], s_qst[NF][NQF];
  __shared__ double s_wm[NF][NQF];  // unloading history of the face points (0: none)
  __shared__ double s_un[NF][BU], s_gln[NF][NF][DIM];
  __shared__ double s_n[NF][DIM], s_area[NF], s_bh[NF], s_ginv[NF][NG > 0 ? NG : 1];
  __shared__ double s_pv[NF][NNF];

  const double det = kp.m.detabs[e];
  // ---- element data and the ids of its interface elements ----------------
  if (tid < NF * DIM) s_gl[tid / DIM][tid % DIM] = kp.m.gl[e * NF * DIM + tid];
  for (int r = tid; r < BU; r += NT) s_ue[r] = u[e * BU + r];
  if (tid < NF) {
    s_f[tid] = kp.m.fid[e * NF + tid];
    s_nb[tid] = kp.m.nbr[e * NF + tid];
  }
  __syncthreads();
  asm volatile("" : "+v"(tid));

  // ---- neighbour and interface data of all faces; bulk shape gradients ----
  for (int t = tid; t < NF * BU; t += NT) {
    const int lf = t / BU, r = t % BU;
    if (s_f[lf] >= 0) s_un[lf][r] = u[(int64_t)s_nb[lf] * BU + r];
  }
  for (int t = tid; t < NF * NF * DIM; t += NT) {
    const int lf = t / (NF * DIM), k = t % (NF * DIM);
    if (s_f[lf] >= 0) s_gln[lf][k / DIM][k % DIM] = kp.m.gl[(int64_t)s_nb[lf] * NF * DIM + k];
  }
  for (int t = tid; t < NF * NQF; t += NT) {
    const int lf = t / NQF, q = t % NQF;
    if (s_f[lf] >= 0) {
      s_qst[lf][q] = kp.m.qp_state[(int64_t)s_f[lf] * NQF + q];
      s_wm[lf][q] = kp.wmax ? kp.wmax[(int64_t)s_f[lf] * NQF + q] : 0.0;
    }
  }
  if (tid < NF) {
    const int32_t f = s_f[tid];
    if (f >= 0) {
      const bool minus = (kp.m.face_em[f] == (int32_t)e);
      s_minus[tid] = minus;
      s_area[tid] = kp.m.area[f];
      s_bh[tid] = kp.b_stab / kp.m.hf[f];
      s_beta[tid] = kp.m.beta[f];
      s_slot[tid] = kp.m.slot[f];
      for (int c = 0; c < DIM; ++c) {
        s_n[tid][c] = kp.m.normal[(int64_t)f * DIM + c];
        const int32_t pm = kp.m.fperm_m[(int64_t)f * DIM + c], pp = kp.m.fperm_p[(int64_t)f * DIM + c];
        s_pe[tid][c] = minus ? pm : pp;
        s_pn[tid][c] = minus ? pp : pm;
      }
      for (int c = 0; c < NG; ++c) s_ginv[tid][c] = kp.m.ginv[(int64_t)f * NG + c];
    }
  }
  for (int t = tid; t < NQV * NN; t += NT) {
    const int q = t / NN, a = t % NN;
    int i, j;
    double c1, c2;
    Lag<DIM, ORDER>::node_form(a, i, j, c1, c2);
    const double li = rt.vq_lam[q][i], lj = rt.vq_lam[q][j];
    for (int x = 0; x < DIM; ++x)
      s_gphE[q][a][x] = c1 * (lj * s_gl[i][x] + li * s_gl[j][x]) + c2 * s_gl[i][x];
  }
  __syncthreads();
  asm volatile("" : "+v"(tid));

  // ---- bulk term; pressures of the fluid faces ----------------------------
  for (int t = tid; t < NF * NNF; t += NT) {
    const int lf = t / NNF, k = t % NNF;
    if (s_f[lf] >= 0 && s_beta[lf])
      s_pv[lf][k] = p[kp.m.face_pn[(int64_t)s_slot[lf] * NNF + k]];
  }
  for (int t = tid; t < NQV * DIM * DIM; t += NT) {
    const int q = t / (DIM * DIM), i = (t / DIM) % DIM, x = t % DIM;
    double g = 0.0;
    for (int b = 0; b < NN; ++b) g += s_ue[b * DIM + i] * s_gphE[q][b][x];
    s_gu[q][i][x] = g;
  }
  for (int t = tid; t < NN * NN; t += NT) {
    const int a = t / NN, b = t % NN;
    double Pm[DIM][DIM];
    for (int x = 0; x < DIM; ++x)
      for (int y = 0; y < DIM; ++y) Pm[x][y] = 0.0;
    for (int q = 0; q < NQV; ++q) {
      const double wq = rt.vq_w[q] * det;
      for (int x = 0; x < DIM; ++x)
        for (int y = 0; y < DIM; ++y) Pm[x][y] += wq * s_gphE[q][a][x] * s_gphE[q][b][y];
    }
    double tr = 0.0;
    for (int x = 0; x < DIM; ++x) tr += Pm[x][x];
    for (int i = 0; i < DIM; ++i)
      for (int j = 0; j < DIM; ++j)
        s_diag[(b * DIM + j) * BU + a * DIM + i] =
            lam * Pm[i][j] + G * Pm[j][i] + (i == j ? G * tr : 0.0);
  }
  // zero this element's coupling strips (owned by this workgroup)
  const int64_t sp0 = kp.m.sp_ptr[e], sp1 = kp.m.sp_ptr[e + 1];
  for (int r = tid; r < BU; r += NT)
    for (int64_t k = sp0; k < sp1; ++k) {
      Bs[k * BU + r] = 0.0;
      Cs[k * BU + r] = 0.0;
    }
  __syncthreads();
  asm volatile("" : "+v"(tid));
  for (int r = tid; r < BU; r += NT) {
    const int a = r / DIM, i = r % DIM;
    double acc = 0.0;
    for (int q = 0; q < NQV; ++q) {
      double tr = 0.0;
      for (int x = 0; x < DIM; ++x) tr += s_gu[q][x][x];
      double sn = 0.0;
      for (int x = 0; x < DIM; ++x) {
        const double sig = G * (s_gu[q][i][x] + s_gu[q][x][i]) + (i == x ? lam * tr : 0.0);
        sn += sig * s_gphE[q][a][x];
      }
      acc += rt.vq_w[q] * det * sn;
    }
    s_R[r] = acc;
  }
  __syncthreads();
  asm volatile("" : "+v"(tid));

  const uint32_t clamp = kp.m.clamp[e];

  // ---- interface elements -----------------------------------------------
  // Four phases per face: shape functions of both elements at the face
  // points; jump and averaged gradient; traction, tangent and fluid
  // coefficients per point; then residual rows, coupling strips and both
  // blocks (each thread forms the moments of one test/trial node pair and
  // expands them).  The last phase reads only what the next face's first two
  // phases do not write (s_phE, s_phN, s_gphE, s_gphN are read there, so the
  // next face's first phase waits at the barrier that closes this one).
#pragma unroll 1
  for (int lf = 0; lf < NF; ++lf) {
    const int32_t f = s_f[lf];
    if (f < 0) continue;  // boundary facet: clamped rows or zero traction
    int ft = tid;
    asm volatile("" : "+v"(ft));
    const double sgE = s_minus[lf] ? -1.0 : 1.0, sgN = -sgE;
    const double area = s_area[lf];
    const double bh = s_bh[lf];
    const double kc = bh * (lam + 2.0 * G);
    const int beta = s_beta[lf];
    const double *nrm = s_n[lf];
    // shape functions of both elements at the face points
    for (int t = ft; t < 2 * NQF * NN; t += NT) {
      const int side = t / (NQF * NN), q = (t / NN) % NQF, a = t % NN;
      int i, j;
      double c1, c2;
      Lag<DIM, ORDER>::node_form(a, i, j, c1, c2);
      // barycentrics of nodes i and j at the point: face vertex k of the
      // point's rule sits at local vertex perm[k]; the opposite vertex is 0
      const int *perm = side == 0 ? s_pe[lf] : s_pn[lf];
      double li = 0.0, lj = 0.0;
      for (int k = 0; k < DIM; ++k) {
        const double mu = rt.fq_mu[q][k];
        li = perm[k] == i ? mu : li;
        lj = perm[k] == j ? mu : lj;
      }
      const double(*gl)[DIM] = side == 0 ? s_gl : s_gln[lf];
      const double ph = c1 * li * lj + c2 * li;
      double gn = 0.0;
      for (int x = 0; x < DIM; ++x) {
        const double g = c1 * (lj * gl[i][x] + li * gl[j][x]) + c2 * gl[i][x];
        if (side == 0) s_gphE[q][a][x] = g; else s_gphN[q][a][x] = g;
        gn += g * nrm[x];
      }
      if (side == 0) { s_phE[q][a] = ph; s_gnE[q][a] = gn; } else { s_phN[q][a] = ph; s_gnN[q][a] = gn; }
    }
    __syncthreads();
    asm volatile("" : "+v"(ft));
    // jump and averaged displacement gradient at the points, one entry per thread
    const double *un = s_un[lf];
    for (int t = ft; t < NQF * DIM * (DIM + 1); t += NT) {
      const int q = t / (DIM * (DIM + 1)), i = (t / (DIM + 1)) % DIM, x = t % (DIM + 1);
      double acc;
      if (x == DIM) {
        double a0 = 0.0, a1 = 0.0;
        for (int a = 0; a < NN; ++a) {
          a0 += s_phE[q][a] * s_ue[a * DIM + i];
          a1 += s_phN[q][a] * un[a * DIM + i];
        }
        acc = sgE * a0 + sgN * a1;  // u+ - u-
      } else {
        double b0 = 0.0;
        for (int a = 0; a < NN; ++a)
          b0 += s_ue[a * DIM + i] * s_gphE[q][a][x] + un[a * DIM + i] * s_gphN[q][a][x];
        acc = 0.5 * b0;  // average of the two sides' displacement gradients
      }
      s_gj[q][i][x] = acc;
    }
    __syncthreads();
    asm volatile("" : "+v"(ft));
    // per point: traction tau, interface-law tangent, weight; on fluid faces
    // the coefficients of the C strips, s_p (K'(w) grad p . grad eta_k + eta_k / dt)
    for (int q = ft; q < NQF; q += NT) {
      double tr = 0.0, w = 0.0;
      for (int x = 0; x < DIM; ++x) {
        tr += s_gj[q][x][x];
        w += s_gj[q][x][DIM] * nrm[x];
      }
      const int st = s_qst[lf][q];
      const double al = st > 0 ? 1.0 : 0.0;
      double T, dT;
      traction_law(st, w, P.sigma_c, P.delta_c, kc, s_wm[lf][q], T, dT);
      double ph_p = 0.0;
      double gp[DIM - 1];
      for (int s2 = 0; s2 < DIM - 1; ++s2) gp[s2] = 0.0;
      if (beta) {
        double mu_[DIM];
        for (int k = 0; k < DIM; ++k) mu_[k] = rt.fq_mu[q][k];
        for (int k = 0; k < NNF; ++k) {
          const double pk = s_pv[lf][k];
          double dmu[DIM];
          Lag<DIM - 1, ORDER>::dphi_one(k, mu_, dmu);
          ph_p += Lag<DIM - 1, ORDER>::phi_one(k, mu_) * pk;
          for (int s2 = 0; s2 < DIM - 1; ++s2) gp[s2] += (dmu[s2 + 1] - dmu[0]) * pk;
        }
        const double wp = w > 0.0 ? w : 0.0;
        const double dK = 3.0 * wp * wp / (12.0 * P.mu);
        for (int k = 0; k < NNF; ++k) {
          double dmu[DIM];
          Lag<DIM - 1, ORDER>::dphi_one(k, mu_, dmu);
          const double eta = Lag<DIM - 1, ORDER>::phi_one(k, mu_);
          double gg = 0.0;
          for (int s2 = 0; s2 < DIM - 1; ++s2)
            for (int t2 = 0; t2 < DIM - 1; ++t2)
              gg += gp[s2] * s_ginv[lf][s2 * (DIM - 1) + t2] * (dmu[t2 + 1] - dmu[0]);
          s_eta[q][k] = eta;
          s_fc[q][k] = P.s_p * (dK * gg + eta / P.dt);
        }
      }
      for (int i = 0; i < DIM; ++i) {
        double sn = 0.0;  // <sigma> n, component i (sigma is linear in grad u)
        for (int x = 0; x < DIM; ++x) {
          const double sa = G * (s_gj[q][i][x] + s_gj[q][x][i]) + (i == x ? lam * tr : 0.0);
          sn += sa * nrm[x];
        }
        const double cj = G * s_gj[q][i][DIM] + (lam + G) * nrm[i] * w;
        s_tau[q][i] = (1.0 - al) * (sn + bh * cj) + al * T * nrm[i] - (beta ? ph_p * nrm[i] : 0.0);
      }
      const double W = rt.fq_w[q] * area;
      s_W[q] = W;
      s_c1[q] = W * sgE * (1.0 - al);
      s_c4[q] = W * sgE * al * dT;
    }
    __syncthreads();
    asm volatile("" : "+v"(ft));
    // residual of this element's test functions (c_qa = W_q s_e phi^e_a)
    for (int r = ft; r < BU; r += NT) {
      const int a = r / DIM, i = r % DIM;
      double acc = 0.0;
      for (int q = 0; q < NQF; ++q) acc += s_W[q] * sgE * s_phE[q][a] * s_tau[q][i];
      s_R[r] += acc;
    }
    // coupling strips: B (d R_u / d p) and C (d R_p / d u_e) of this face
    if (beta) {
      for (int t = ft; t < BU * NNF; t += NT) {
        const int r = t % BU, k = t / BU;
        const int a = r / DIM, i = r % DIM;
        const int32_t ix = kp.m.fs_idx[((int64_t)e * NF + lf) * NNF + k];
        double bv = 0.0, cv = 0.0;
        for (int q = 0; q < NQF; ++q) {
          const double ca = s_W[q] * sgE * s_phE[q][a];
          bv -= ca * s_eta[q][k] * nrm[i];
          cv += s_W[q] * s_fc[q][k] * sgE * s_phE[q][a] * nrm[i];
        }
        Bs[(int64_t)ix * BU + r] += bv;
        if (!kp.freeze_p) Cs[(int64_t)ix * BU + r] += cv;
      }
    }
    // self block (into the diagonal) and the off-diagonal block: per test node
    // a / trial node b the moments over the points of both trial sides
    //   M1[x] = sum_q c_qa (1-alpha_q) dphi_b/dx_x,  M2 = sum_q c_qa (1-alpha_q) grad phi_b . n,
    //   M3    = sum_q c_qa (1-alpha_q) phi_b,         M4 = sum_q c_qa alpha_q T'(w_q) phi_b,
    // expanded to the 3x3 (2x2) node block; the off-diagonal block goes
    // straight to memory (for each (b, j) the threads of consecutive a write
    // one run of BU values)
    double *Aoff = A + (int64_t)kp.m.blk_of[e * NF + lf] * BU * BU;
    for (int t = ft; t < NN * NN; t += NT) {
      const int b = t / NN, a = t % NN;
      double M[2][DIM + 3];
      for (int side = 0; side < 2; ++side)
        for (int x = 0; x < DIM + 3; ++x) M[side][x] = 0.0;
#pragma unroll 3
      for (int q = 0; q < NQF; ++q) {
        const double pa = s_phE[q][a];
        const double c1 = s_c1[q] * pa, c4 = s_c4[q] * pa;
        for (int x = 0; x < DIM; ++x) {
          M[0][x] += c1 * s_gphE[q][b][x];
          M[1][x] += c1 * s_gphN[q][b][x];
        }
        M[0][DIM] += c1 * s_gnE[q][b];
        M[1][DIM] += c1 * s_gnN[q][b];
        const double pe = s_phE[q][b], pn = s_phN[q][b];
        M[0][DIM + 1] += c1 * pe;
        M[1][DIM + 1] += c1 * pn;
        M[0][DIM + 2] += c4 * pe;
        M[1][DIM + 2] += c4 * pn;
      }
      // B[a i][b j] = n_i (lam/2 M1_j) + n_j (G/2 M1_i) + n_i n_j s1 + d_ij s2 with
      // s1 = s_t ((b/h)(lam+G) M3 + M4), s2 = s_t (b/h) G M3 + G/2 M2
      // (the expansion of lam/2 n_i M1_j + G/2 n_j M1_i + G/2 d_ij M2
      //  + (b/h) s_t Chat_ij M3 + s_t n_i n_j M4, Chat = G I + (lam+G) n n)
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const double sg = side == 0 ? sgE : sgN;
        const double s1 = sg * (bh * (lam + G) * M[side][DIM + 1] + M[side][DIM + 2]);
        const double s2 = sg * bh * G * M[side][DIM + 1] + 0.5 * G * M[side][DIM];
        double pl[DIM], pg[DIM];
        for (int x = 0; x < DIM; ++x) {
          pl[x] = 0.5 * lam * M[side][x];
          pg[x] = 0.5 * G * M[side][x];
        }
        for (int j = 0; j < DIM; ++j)
          for (int i = 0; i < DIM; ++i) {
            double v = nrm[i] * pl[j] + nrm[j] * pg[i] + nrm[i] * nrm[j] * s1;
            if (i == j) v += s2;
            const int r = a * DIM + i;
            const int idx = (b * DIM + j) * BU + r;
            if (side == 0) s_diag[idx] += v;
            else Aoff[idx] = ((clamp >> r) & 1u) ? 0.0 : v;
          }
      }
    }
    __syncthreads();
  }

  // ---- strong Dirichlet rows and write-back ------------------------------
  double *Ad = A + kp.m.blk_ptr[e] * BU * BU;
  for (int idx = tid; idx < BU * BU; idx += NT) {
    const int c = idx / BU, r = idx % BU;
    double v = s_diag[idx];
    if ((clamp >> r) & 1u) v = (r == c) ? 1.0 : 0.0;
    Ad[idx] = v;
  }
  for (int r = tid; r < BU; r += NT) {
    const bool cl = (clamp >> r) & 1u;
    R[e * BU + r] = cl ? s_ue[r] : s_R[r];
    if (cl)
      for (int64_t k = sp0; k < sp1; ++k) Bs[k * BU + r] = 0.0;
  }
}

// Persistent form: a grid sized to the workgroups the chip holds at once
// walks the element list (all instances of the batch, concatenated), one
// element per workgroup at a time; the barrier at the end of each element
// keeps the next element's LDS writes behind this one's last reads.  The
// quadrature rules of the context are staged in LDS once per workgroup.
template <int DIM, int ORDER, int NT>
__global__ __launch_bounds__(NT, 3) void k_assemble(KParams kp, const int32_t *__restrict__ elist,
                                                 int64_t n_items, const double *__restrict__ u,
                                                 const double *__restrict__ p,
                                                 const double *__restrict__ w_old,
                                                 double *__restrict__ A, double *__restrict__ R,
                                                 double *__restrict__ Bs,
                                                 double *__restrict__ Cs) {
  __shared__ RuleTables s_rt;
  {
    const int *src = reinterpret_cast<const int *>(kp.rt);
    int *dst = reinterpret_cast<int *>(&s_rt);
    for (int i = threadIdx.x; i < (int)(sizeof(RuleTables) / sizeof(int)); i += NT) dst[i] = src[i];
  }
  __syncthreads();
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int64_t e = elist ? (int64_t)elist[it] : it;
    assemble_element<DIM, ORDER, NT>(kp, s_rt, e, u, p, w_old, A, R, Bs, Cs);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Fluid rows: R_p and the dense row of D, one thread per pressure node
// ---------------------------------------------------------------------------
template <int DIM, int ORDER>
__device__ __forceinline__ void fluid_row(const KParams &kp, const int64_t i,
                                          const double *__restrict__ u,
                                          const double *__restrict__ p,
                                          const double *__restrict__ w_old,
                                          double *__restrict__ R, double *__restrict__ D) {
  using C = Cfg<DIM, ORDER>;
  constexpr int NN = C::NN, BU = C::BU, NQF = C::NQF, NNF = C::NNF;
  __shared__ double srow[kMaxPressureBlock];  // the dense row of D being summed
  __shared__ double s_r[64], s_d[64][NNF];
  __shared__ int s_c[64][NNF];
  const int lane = threadIdx.x;
  const int b = kp.pinst[i];
  const InstPar P = kp.ip[b];
  const int32_t p0 = kp.poff[b];
  const int nb = kp.poff[b + 1] - p0;
  double *Drow = D + kp.doff[b] + (i - p0) * (int64_t)nb;
  if (kp.freeze_p) {  // pressure held at its current value: dp = 0
    for (int j = lane; j < nb; j += 64) Drow[j] = (j == i - p0) ? 1.0 : 0.0;
    if (lane == 0) R[kp.s.n_u + i] = 0.0;
    return;
  }
  for (int j = lane; j < nb; j += 64) srow[j] = 0.0;
  const int32_t t0 = kp.m.pf_ptr[i];
  const int nfq = (kp.m.pf_ptr[i + 1] - t0) * NQF;
  double Ri = 0.0;  // lane NNF sums the residual terms
  for (int base = 0; base < nfq; base += 64) {
    // one (face, point) term per lane: its residual part and its NNF
    // contributions to the row of D
    const int idx = base + lane;
    if (idx < nfq) {
      const int32_t t = t0 + idx / NQF;
      const int q = idx % NQF;
      const int32_t fa = kp.m.pf_fa[t], kk = kp.m.pf_k[t];
      const int32_t f = kp.m.act_face[fa];
      const int32_t em = kp.m.face_em[f], ep = kp.m.face_ep[f];
      double n[DIM];
      for (int x = 0; x < DIM; ++x) n[x] = kp.m.normal[(int64_t)f * DIM + x];
      const double area = kp.m.area[f];
      double gi[(DIM - 1) * (DIM - 1)];
      for (int s2 = 0; s2 < (DIM - 1) * (DIM - 1); ++s2) gi[s2] = kp.m.ginv[(int64_t)f * (DIM - 1) * (DIM - 1) + s2];
      int32_t pn[NNF];
      for (int k = 0; k < NNF; ++k) pn[k] = kp.m.face_pn[(int64_t)fa * NNF + k];
      double lm[DIM + 1], lp[DIM + 1];
      for (int k = 0; k <= DIM; ++k) lm[k] = lp[k] = 0.0;
      for (int k = 0; k < DIM; ++k) {
        lm[kp.m.fperm_m[(int64_t)f * DIM + k]] = kp.rt->fq_mu[q][k];
        lp[kp.m.fperm_p[(int64_t)f * DIM + k]] = kp.rt->fq_mu[q][k];
      }
      double w = 0.0;
      for (int x = 0; x < DIM; ++x) {
        double um = 0.0, up = 0.0;
        for (int a = 0; a < NN; ++a) {
          um += Lag<DIM, ORDER>::phi_one(a, lm) * u[(int64_t)em * BU + a * DIM + x];
          up += Lag<DIM, ORDER>::phi_one(a, lp) * u[(int64_t)ep * BU + a * DIM + x];
        }
        w += (up - um) * n[x];
      }
      const double wp = w > 0.0 ? w : 0.0;
      const double K = wp * wp * wp / (12.0 * P.mu);
      double mu_[DIM];
      for (int k = 0; k < DIM; ++k) mu_[k] = kp.rt->fq_mu[q][k];
      double gp[DIM - 1];
      for (int s2 = 0; s2 < DIM - 1; ++s2) gp[s2] = 0.0;
      for (int k = 0; k < NNF; ++k) {
        double dmu[DIM];
        Lag<DIM - 1, ORDER>::dphi_one(k, mu_, dmu);
        for (int s2 = 0; s2 < DIM - 1; ++s2) gp[s2] += (dmu[s2 + 1] - dmu[0]) * p[pn[k]];
      }
      double dk[DIM];
      Lag<DIM - 1, ORDER>::dphi_one(kk, mu_, dk);
      const double etak = Lag<DIM - 1, ORDER>::phi_one(kk, mu_);
      const double W = kp.rt->fq_w[q] * area;
      double gpg = 0.0;
      for (int s2 = 0; s2 < DIM - 1; ++s2)
        for (int t2 = 0; t2 < DIM - 1; ++t2) gpg += gp[s2] * gi[s2 * (DIM - 1) + t2] * (dk[t2 + 1] - dk[0]);
      const double wo = w_old[(int64_t)f * NQF + q];
      s_r[lane] = P.s_p * W * (K * gpg + (w - wo) / P.dt * etak);
      for (int l = 0; l < NNF; ++l) {
        double dl[DIM];
        Lag<DIM - 1, ORDER>::dphi_one(l, mu_, dl);
        double gg = 0.0;
        for (int s2 = 0; s2 < DIM - 1; ++s2)
          for (int t2 = 0; t2 < DIM - 1; ++t2) gg += (dl[s2 + 1] - dl[0]) * gi[s2 * (DIM - 1) + t2] * (dk[t2 + 1] - dk[0]);
        s_d[lane][l] = P.s_p * W * K * gg;
        s_c[lane][l] = pn[l] - p0;
      }
    }
    __syncthreads();
    // sum in (face, point) order: at each term the NNF lanes touch NNF
    // distinct columns (the face's pressure nodes), so every column and the
    // residual receive their terms in the same order as a serial loop
    const int cnt = min(64, nfq - base);
    if (lane < NNF) {
      for (int k = 0; k < cnt; ++k) srow[s_c[k][lane]] += s_d[k][lane];
    } else if (lane == NNF) {
      for (int k = 0; k < cnt; ++k) Ri += s_r[k];
    }
    __syncthreads();
  }
  for (int j = lane; j < nb; j += 64) Drow[j] = srow[j];
  if (lane == NNF) {
    for (int64_t s2 = 0; s2 < kp.s.n_src; ++s2)
      if (kp.m.src_node[s2] == i) Ri -= P.s_p * kp.m.src_q0[s2];
    R[kp.s.n_u + i] = Ri;
  }
}

// Persistent form over the pressure nodes of the batch, as for k_assemble.
template <int DIM, int ORDER>
__global__ __launch_bounds__(64) void k_fluid_rows(KParams kp, const double *__restrict__ u,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ w_old,
                                                   double *__restrict__ R, double *__restrict__ D) {
  for (int64_t i = blockIdx.x; i < kp.s.n_p; i += gridDim.x) {
    fluid_row<DIM, ORDER>(kp, i, u, p, w_old, R, D);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Opening w = [[u]] . n at every face point
// ---------------------------------------------------------------------------
template <int DIM, int ORDER>
__global__ void k_opening(KParams kp, const double *__restrict__ u, double *__restrict__ w) {
  using C = Cfg<DIM, ORDER>;
  constexpr int NN = C::NN, BU = C::BU, NQF = C::NQF;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= kp.s.nf * NQF) return;
  const int64_t f = t / NQF;
  const int q = (int)(t % NQF);
  const int32_t em = kp.m.face_em[f], ep = kp.m.face_ep[f];
  double lm[DIM + 1], lp[DIM + 1];
  for (int k = 0; k <= DIM; ++k) lm[k] = lp[k] = 0.0;
  for (int k = 0; k < DIM; ++k) {
    lm[kp.m.fperm_m[f * DIM + k]] = kp.rt->fq_mu[q][k];
    lp[kp.m.fperm_p[f * DIM + k]] = kp.rt->fq_mu[q][k];
  }
  double phm[NN], php[NN];
  Lag<DIM, ORDER>::phi(lm, phm);
  Lag<DIM, ORDER>::phi(lp, php);
  double acc = 0.0;
  for (int x = 0; x < DIM; ++x) {
    double um = 0.0, up = 0.0;
    for (int a = 0; a < NN; ++a) {
      um += phm[a] * u[(int64_t)em * BU + a * DIM + x];
      up += php[a] * u[(int64_t)ep * BU + a * DIM + x];
    }
    acc += (up - um) * kp.m.normal[f * DIM + x];
  }
  w[t] = acc;
}

// normal traction the DG method exchanges at every face point, the flux of
// the consistency and stabilisation terms: t.n = n.{sigma(u)} n +
// (b/h_f)(lambda + 2G) [[u]].n (Chat(n) n = (lambda + 2G) n); one thread per
// (face, point)
template <int DIM, int ORDER>
__global__ void k_face_traction(KParams kp, const double *__restrict__ u, double *__restrict__ tn) {
  using C = Cfg<DIM, ORDER>;
  constexpr int NN = C::NN, BU = C::BU, NQF = C::NQF;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= kp.s.nf * NQF) return;
  const int64_t f = t / NQF;
  const int q = (int)(t % NQF);
  const int32_t es[2] = {kp.m.face_em[f], kp.m.face_ep[f]};
  const int32_t *perm[2] = {kp.m.fperm_m, kp.m.fperm_p};
  const InstPar P = kp.ip[kp.einst[es[0]]];
  double n[DIM];
  for (int x = 0; x < DIM; ++x) n[x] = kp.m.normal[f * DIM + x];
  double snn = 0.0, w = 0.0;
  for (int side = 0; side < 2; ++side) {
    const int64_t e = es[side];
    double lam[DIM + 1];
    for (int k = 0; k <= DIM; ++k) lam[k] = 0.0;
    for (int k = 0; k < DIM; ++k) lam[perm[side][f * DIM + k]] = kp.rt->fq_mu[q][k];
    const double *gl = kp.m.gl + e * (DIM + 1) * DIM;
    double gu[DIM][DIM], uv[DIM];
    for (int i = 0; i < DIM; ++i) {
      uv[i] = 0.0;
      for (int x = 0; x < DIM; ++x) gu[i][x] = 0.0;
    }
    for (int a = 0; a < NN; ++a) {
      double dl[DIM + 1];
      Lag<DIM, ORDER>::dphi_one(a, lam, dl);
      double g[DIM];
      for (int x = 0; x < DIM; ++x) {
        g[x] = 0.0;
        for (int k = 0; k <= DIM; ++k) g[x] += dl[k] * gl[k * DIM + x];
      }
      const double ph = Lag<DIM, ORDER>::phi_one(a, lam);
      for (int i = 0; i < DIM; ++i) {
        const double ua = u[e * BU + a * DIM + i];
        uv[i] += ph * ua;
        for (int x = 0; x < DIM; ++x) gu[i][x] += ua * g[x];
      }
    }
    double tr = 0.0, nen = 0.0;
    for (int i = 0; i < DIM; ++i) {
      tr += gu[i][i];
      for (int x = 0; x < DIM; ++x) nen += n[i] * 0.5 * (gu[i][x] + gu[x][i]) * n[x];
    }
    snn += 0.5 * (P.lam * tr + 2.0 * P.G * nen);
    for (int i = 0; i < DIM; ++i) w += (side ? uv[i] : -uv[i]) * n[i];
  }
  tn[t] = snn + kp.b_stab / kp.m.hf[f] * (P.lam + 2.0 * P.G) * w;
}

// activation checks on a converged state, one thread per face: an intact
// point whose DG normal traction exceeds sigma_c becomes cohesive (state 1);
// a face without fluid whose points are all cohesive or traction-free becomes
// a fluid face once its opening exceeds delta_c at any point
template <int NQF>
__global__ void k_activation(KParams kp, const double *__restrict__ tn, const double *__restrict__ w,
                             uint8_t *__restrict__ qp_out, uint8_t *__restrict__ beta_out) {
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= kp.s.nf) return;
  const InstPar P = kp.ip[kp.einst[kp.m.face_em[f]]];
  bool all_open = true, wide = false;
  for (int q = 0; q < NQF; ++q) {
    const int64_t t = f * NQF + q;
    uint8_t st = kp.m.qp_state[t];
    if (st == 0 && tn[t] > P.sigma_c) st = 1;
    qp_out[t] = st;
    all_open = all_open && st >= 1;
    wide = wide || w[t] > P.delta_c;
  }
  beta_out[f] = (kp.m.beta[f] || (all_open && wide)) ? 1 : 0;
}

// crack volume of each instance: out[b] = sum over its fluid faces and points of W_q w_q
template <int DIM, int ORDER>
__global__ __launch_bounds__(256) void k_fluid_volume(KParams kp, const double *__restrict__ u,
                                                      double *__restrict__ out) {
  using C = Cfg<DIM, ORDER>;
  constexpr int NN = C::NN, BU = C::BU, NQF = C::NQF;
  __shared__ double sm[256];
  const int b = blockIdx.x;
  double acc = 0.0;
  const int64_t t0 = (int64_t)kp.aoff[b] * NQF, t1 = (int64_t)kp.aoff[b + 1] * NQF;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += 256) {
    const int64_t f = kp.m.act_face[t / NQF];
    const int q = (int)(t % NQF);
    const int32_t em = kp.m.face_em[f], ep = kp.m.face_ep[f];
    double lm[DIM + 1], lp[DIM + 1];
    for (int k = 0; k <= DIM; ++k) lm[k] = lp[k] = 0.0;
    for (int k = 0; k < DIM; ++k) {
      lm[kp.m.fperm_m[f * DIM + k]] = kp.rt->fq_mu[q][k];
      lp[kp.m.fperm_p[f * DIM + k]] = kp.rt->fq_mu[q][k];
    }
    double w = 0.0;
    for (int x = 0; x < DIM; ++x) {
      double um = 0.0, up = 0.0;
      for (int a = 0; a < NN; ++a) {
        um += Lag<DIM, ORDER>::phi_one(a, lm) * u[(int64_t)em * BU + a * DIM + x];
        up += Lag<DIM, ORDER>::phi_one(a, lp) * u[(int64_t)ep * BU + a * DIM + x];
      }
      w += (up - um) * kp.m.normal[f * DIM + x];
    }
    acc += kp.rt->fq_w[q] * kp.m.area[f] * w;
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = sm[0];
}

// max of w over the face points of each instance's fluid faces: out[b]
__global__ void k_wmax(KParams kp, const double *__restrict__ w, double *out) {
  __shared__ double sm[256];
  const int nq = kp.s.nqf;
  const int b = blockIdx.x;
  double mx = -1e300;
  for (int64_t t = (int64_t)kp.aoff[b] * nq + threadIdx.x; t < (int64_t)kp.aoff[b + 1] * nq; t += blockDim.x) {
    const int32_t f = kp.m.act_face[t / nq];
    mx = fmax(mx, w[(int64_t)f * nq + t % nq]);
  }
  sm[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = sm[0];
}

template <int DIM, int ORDER>
static hipError_t assemble_impl(const KParams &kp, const double *u, const double *p,
                                const double *w_old, double *A, double *R, double *Bs,
                                double *Cs, double *D, const int32_t *elist, int64_t n_el,
                                hipStream_t st) {
  constexpr int NT = (Cfg<DIM, ORDER>::BU >= 24) ? 128 : 64;
  static ResidentGrid g_el, g_fl;
  if (n_el) {
    unsigned g = 0;
    hipError_t err = g_el.size((const void *)k_assemble<DIM, ORDER, NT>, NT, n_el, &g);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_assemble<DIM, ORDER, NT>), dim3(g), dim3(NT), 0, st, kp, elist, n_el, u,
                       p, w_old, A, R, Bs, Cs);
  }
  if (kp.s.n_p) {
    unsigned g = 0;
    hipError_t err = g_fl.size((const void *)k_fluid_rows<DIM, ORDER>, 64, kp.s.n_p, &g);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_fluid_rows<DIM, ORDER>), dim3(g), dim3(64), 0, st, kp, u, p, w_old, R, D);
  }
  return hipGetLastError();
}

hipError_t launch_assemble(const KParams &kp, const double *u, const double *p,
                           const double *w_old, double *A, double *R, double *Bs, double *Cs,
                           double *D, const int32_t *elist, int64_t n_el, hipStream_t st) {
  const int d = kp.s.dim, o = kp.s.order;
  if (!elist) n_el = kp.s.ne;
  if (d == 2 && o == 1) return assemble_impl<2, 1>(kp, u, p, w_old, A, R, Bs, Cs, D, elist, n_el, st);
  if (d == 2 && o == 2) return assemble_impl<2, 2>(kp, u, p, w_old, A, R, Bs, Cs, D, elist, n_el, st);
  if (d == 3 && o == 1) return assemble_impl<3, 1>(kp, u, p, w_old, A, R, Bs, Cs, D, elist, n_el, st);
  if (d == 3 && o == 2) return assemble_impl<3, 2>(kp, u, p, w_old, A, R, Bs, Cs, D, elist, n_el, st);
  return hipErrorInvalidValue;
}

hipError_t launch_opening(const KParams &kp, const double *u, double *w, hipStream_t st) {
  const int64_t n = kp.s.nf * kp.s.nqf;
  if (!n) return hipSuccess;
  dim3 g((unsigned)((n + 127) / 128)), b(128);
  const int d = kp.s.dim, o = kp.s.order;
  if (d == 2 && o == 1) hipLaunchKernelGGL((k_opening<2, 1>), g, b, 0, st, kp, u, w);
  else if (d == 2 && o == 2) hipLaunchKernelGGL((k_opening<2, 2>), g, b, 0, st, kp, u, w);
  else if (d == 3 && o == 1) hipLaunchKernelGGL((k_opening<3, 1>), g, b, 0, st, kp, u, w);
  else hipLaunchKernelGGL((k_opening<3, 2>), g, b, 0, st, kp, u, w);
  return hipGetLastError();
}

hipError_t launch_face_traction(const KParams &kp, const double *u, double *tn, hipStream_t st) {
  const int64_t n = kp.s.nf * kp.s.nqf;
  if (!n) return hipSuccess;
  dim3 g((unsigned)((n + 127) / 128)), b(128);
  const int d = kp.s.dim, o = kp.s.order;
  if (d == 2 && o == 1) hipLaunchKernelGGL((k_face_traction<2, 1>), g, b, 0, st, kp, u, tn);
  else if (d == 2 && o == 2) hipLaunchKernelGGL((k_face_traction<2, 2>), g, b, 0, st, kp, u, tn);
  else if (d == 3 && o == 1) hipLaunchKernelGGL((k_face_traction<3, 1>), g, b, 0, st, kp, u, tn);
  else hipLaunchKernelGGL((k_face_traction<3, 2>), g, b, 0, st, kp, u, tn);
  return hipGetLastError();
}

hipError_t launch_activation(const KParams &kp, const double *tn, const double *w, uint8_t *qp_out,
                             uint8_t *beta_out, hipStream_t st) {
  if (!kp.s.nf) return hipSuccess;
  dim3 g((unsigned)((kp.s.nf + 127) / 128)), b(128);
  switch (kp.s.nqf) {
    case 2: hipLaunchKernelGGL((k_activation<2>), g, b, 0, st, kp, tn, w, qp_out, beta_out); break;
    case 3: hipLaunchKernelGGL((k_activation<3>), g, b, 0, st, kp, tn, w, qp_out, beta_out); break;
    case 4: hipLaunchKernelGGL((k_activation<4>), g, b, 0, st, kp, tn, w, qp_out, beta_out); break;
    case 9: hipLaunchKernelGGL((k_activation<9>), g, b, 0, st, kp, tn, w, qp_out, beta_out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fluid_volume(const KParams &kp, const double *u, double *partial, double *out,
                               hipStream_t st) {
  (void)partial;
  const int nb = kp.n_inst;
  const int d = kp.s.dim, o = kp.s.order;
  if (d == 2 && o == 1) hipLaunchKernelGGL((k_fluid_volume<2, 1>), dim3(nb), dim3(256), 0, st, kp, u, out);
  else if (d == 2 && o == 2) hipLaunchKernelGGL((k_fluid_volume<2, 2>), dim3(nb), dim3(256), 0, st, kp, u, out);
  else if (d == 3 && o == 1) hipLaunchKernelGGL((k_fluid_volume<3, 1>), dim3(nb), dim3(256), 0, st, kp, u, out);
  else hipLaunchKernelGGL((k_fluid_volume<3, 2>), dim3(nb), dim3(256), 0, st, kp, u, out);
  return hipGetLastError();
}

__global__ void k_max_into(const double *__restrict__ x, double *__restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = fmax(y[i], x[i]);
}

hipError_t launch_max_into(const double *x, double *y, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_max_into, dim3(g), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

hipError_t launch_wmax(const KParams &kp, const double *w, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_wmax, dim3(kp.n_inst), dim3(256), 0, st, kp, w, out);
  return hipGetLastError();
}

}  // namespace hf
