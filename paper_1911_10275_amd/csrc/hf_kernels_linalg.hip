// Linear-algebra kernels for gfx950: block-sparse Jacobian product,
// pressure rows, batched block inverses, the Schur pressure block, and the
// Krylov vector kernels with deterministic two-stage reductions.
//
// Jacobian storage.  Element row e of A is one contiguous "row panel": its
// blocks (diagonal first, then one per interior face in local-face order)
// each stored column-major, so the panel is a column-major bs x (nb*bs)
// matrix.  The product streams each panel with 16-byte loads: a group of L
// lanes reads CH = LA*EL consecutive values per step, and because CH is a
// multiple of bs every lane keeps the same rows at every step; the products
// are summed per lane and combined across lanes in a fixed order at the end.
#include <cmath>

#include "hf_internal.h"

namespace hf {

// ---------------------------------------------------------------------------
// Block-sparse product y = A x (+ B x_p on rows with coupling strips)
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int active_lanes(int L, int EL, int BU) {
  int la = L;
  while (la > 0 && (la * EL) % BU != 0) --la;
  return la;
}

template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int EL = 2;
};
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int EL = 4;
};

template <typename T, int BU>
struct SpmvShape {
  static constexpr int EL = Vec16<T>::EL;
  static constexpr int L = BU >= 24 ? 64 : (BU >= 12 ? 32 : 16);
  static constexpr int LA = active_lanes(L, EL, BU);
  static constexpr int CH = LA * EL;
  static constexpr int RPC = CH / BU;  // columns advanced per step
  static_assert(CH % BU == 0, "chunk must hold whole columns");
};

template <typename T>
__device__ inline T vget(const typename Vec16<T>::type &v, int s);
template <>
__device__ inline double vget<double>(const double2 &v, int s) { return s == 0 ? v.x : v.y; }
template <>
__device__ inline float vget<float>(const float4 &v, int s) {
  return s == 0 ? v.x : (s == 1 ? v.y : (s == 2 ? v.z : v.w));
}

template <typename T, int BU, int NT, bool STRIPS>
__global__ __launch_bounds__(NT) void k_bsr_spmv(
    int64_t ne, const int64_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const T *__restrict__ A, const int64_t *__restrict__ sp_ptr,
    const int32_t *__restrict__ sp_pnode, const T *__restrict__ Bs, const T *__restrict__ x,
    const T *__restrict__ xp, T *__restrict__ y) {
  using S = SpmvShape<T, BU>;
  constexpr int L = S::L, EL = S::EL, LA = S::LA, CH = S::CH, RPC = S::RPC, G = NT / L;
  using V = typename Vec16<T>::type;
  __shared__ T xs[G][5 * BU];
  __shared__ T part[G][CH];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int64_t e = (int64_t)blockIdx.x * G + g;
  int64_t b0 = 0;
  int nb = 0;
  if (e < ne) {
    b0 = blk_ptr[e];
    nb = (int)(blk_ptr[e + 1] - b0);
    for (int t = lane; t < nb * BU; t += L) xs[g][t] = x[(int64_t)blk_col[b0 + t / BU] * BU + t % BU];
  }
  __syncthreads();
  T acc[EL];
#pragma unroll
  for (int s = 0; s < EL; ++s) acc[s] = T(0);
  if (e < ne && lane < LA) {
    const T *panel = A + b0 * BU * BU;
    const int total = nb * BU * BU;
    int colS[EL];
#pragma unroll
    for (int s = 0; s < EL; ++s) colS[s] = (lane * EL + s) / BU;
    int f = lane * EL, cb = 0;
#pragma unroll 4
    for (; f < total; f += CH, cb += RPC) {
      const V v = *(const V *)(panel + f);
#pragma unroll
      for (int s = 0; s < EL; ++s) acc[s] += vget<T>(v, s) * xs[g][cb + colS[s]];
    }
  }
  if (lane < LA) {
#pragma unroll
    for (int s = 0; s < EL; ++s) part[g][lane * EL + s] = acc[s];
  }
  __syncthreads();
  if (e < ne && lane < BU) {
    T sum = T(0);
#pragma unroll
    for (int t = 0; t < RPC; ++t) sum += part[g][lane + BU * t];
    if (STRIPS) {
      for (int64_t k = sp_ptr[e]; k < sp_ptr[e + 1]; ++k) sum += Bs[k * BU + lane] * xp[sp_pnode[k]];
    }
    y[e * BU + lane] = sum;
  }
}

// pressure rows: y_p[i] = sum_strips C x_u + sum_j D_b[i][j] x_p[j] over the dense block
// of the row's instance b (one wave per row)
template <typename T, int BU>
__global__ __launch_bounds__(64) void k_prows(int64_t np, const int32_t *__restrict__ pinst,
                                              const int32_t *__restrict__ poff,
                                              const int64_t *__restrict__ doff,
                                              const int32_t *__restrict__ pc_ptr,
                                              const int32_t *__restrict__ pc_ent,
                                              const int32_t *__restrict__ sp_elem,
                                              const T *__restrict__ Cs, const T *__restrict__ D,
                                              const T *__restrict__ xu, const T *__restrict__ xp,
                                              T *__restrict__ yp) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  double acc = 0.0;
  if (pc_ptr) {
    for (int32_t c = pc_ptr[i]; c < pc_ptr[i + 1]; ++c) {
      const int32_t ent = pc_ent[c];
      const int64_t e = sp_elem[ent];
      if (lane < BU) acc += (double)Cs[(int64_t)ent * BU + lane] * (double)xu[e * BU + lane];
    }
  }
  const int b = pinst[i];
  const int64_t p0 = poff[b], nb = poff[b + 1] - p0;
  const T *Drow = D + doff[b] + (i - p0) * nb;
  for (int64_t j = lane; j < nb; j += 64) acc += (double)Drow[j] * (double)xp[p0 + j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) yp[i] = (T)acc;
}

template <typename T, int BU>
static void spmv_bu(const KParams &kp, const T *A, const T *Bs, const T *Cs, const T *D,
                    const T *x, T *y, hipStream_t st) {
  using S = SpmvShape<T, BU>;
  constexpr int NT = 256, G = NT / S::L;
  const int64_t ne = kp.s.ne;
  if (ne)
    hipLaunchKernelGGL((k_bsr_spmv<T, BU, NT, true>), dim3((unsigned)((ne + G - 1) / G)), dim3(NT), 0, st,
                       ne, kp.m.blk_ptr, kp.m.blk_col, A, kp.m.sp_ptr, kp.m.sp_pnode, Bs, x,
                       x + kp.s.n_u, y);
  if (kp.s.n_p)
    hipLaunchKernelGGL((k_prows<T, BU>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.s.n_p,
                       kp.pinst, kp.poff, kp.doff, kp.m.pc_ptr, kp.m.pc_ent, kp.m.sp_elem, Cs, D, x,
                       x + kp.s.n_u, y + kp.s.n_u);
}

template <typename T>
hipError_t launch_spmv(const KParams &kp, const T *A, const T *Bs, const T *Cs, const T *D,
                       const T *x, T *y, hipStream_t st) {
  switch (kp.s.bu) {
    case 6: spmv_bu<T, 6>(kp, A, Bs, Cs, D, x, y, st); break;
    case 12: spmv_bu<T, 12>(kp, A, Bs, Cs, D, x, y, st); break;
    case 30: spmv_bu<T, 30>(kp, A, Bs, Cs, D, x, y, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_spmv<double>(const KParams &, const double *, const double *,
                                        const double *, const double *, const double *,
                                        double *, hipStream_t);
template hipError_t launch_spmv<float>(const KParams &, const float *, const float *,
                                       const float *, const float *, const float *, float *,
                                       hipStream_t);

// block-Jacobi apply: z_u = blockdiag(inv) r_u (the same streaming kernel on
// the identity block pattern), z_p = S^-1 r_p
template <typename T, int BU>
static void precond_bu(const KParams &kp, const T *inv, const T *Sinv, const T *r, T *z,
                       hipStream_t st, const int64_t *ident_ptr, const int32_t *ident_col) {
  using S = SpmvShape<T, BU>;
  constexpr int NT = 256, G = NT / S::L;
  const int64_t ne = kp.s.ne;
  if (ne)
    hipLaunchKernelGGL((k_bsr_spmv<T, BU, NT, false>), dim3((unsigned)((ne + G - 1) / G)), dim3(NT), 0, st,
                       ne, ident_ptr, ident_col, inv, nullptr, nullptr, nullptr, r, nullptr, z);
  if (kp.s.n_p)
    hipLaunchKernelGGL((k_prows<T, BU>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.s.n_p,
                       kp.pinst, kp.poff, kp.doff, nullptr, nullptr, nullptr, nullptr, Sinv, r,
                       r + kp.s.n_u, z + kp.s.n_u);
}

template <typename T>
hipError_t launch_precond(const KParams &kp, const T *inv, const T *Sinv, const T *r, T *z,
                          hipStream_t st) {
  const int64_t *ip = kp.m.ident_ptr;
  const int32_t *ic = kp.m.ident_col;
  switch (kp.s.bu) {
    case 6: precond_bu<T, 6>(kp, inv, Sinv, r, z, st, ip, ic); break;
    case 12: precond_bu<T, 12>(kp, inv, Sinv, r, z, st, ip, ic); break;
    case 30: precond_bu<T, 30>(kp, inv, Sinv, r, z, st, ip, ic); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_precond<double>(const KParams &, const double *, const double *,
                                           const double *, double *, hipStream_t);
template hipError_t launch_precond<float>(const KParams &, const float *, const float *,
                                          const float *, float *, hipStream_t);

// ---------------------------------------------------------------------------
// Batched inverse of the diagonal element blocks: Gauss-Jordan with partial
// (row) pivoting, one wavefront per block, lane r holds row r in registers.
// Pivot rows are chosen in place (no physical swap); the inverse is read out
// with the column permutation the pivot order implies.
// ---------------------------------------------------------------------------
template <int BU>
__global__ __launch_bounds__(64) void k_blockinv(int64_t ne, const int64_t *__restrict__ blk_ptr,
                                                 const int32_t *__restrict__ einst,
                                                 const double *__restrict__ A,
                                                 double *__restrict__ inv,
                                                 float *__restrict__ inv32, int *flag) {
  const int64_t e = blockIdx.x;
  const int lane = threadIdx.x;
  __shared__ double prow[BU];
  __shared__ int s_pk[BU];
  const double *blk = A + blk_ptr[e] * BU * BU;
  double a[BU];
#pragma unroll
  for (int c = 0; c < BU; ++c) a[c] = lane < BU ? blk[c * BU + lane] : 0.0;
  bool used = lane >= BU;
  int mystep = 0;
#pragma unroll
  for (int k = 0; k < BU; ++k) {
    // NaN ranks above every number so that it is picked and reported
    double v = used ? -1.0 : (isnan(a[k]) ? INFINITY : fabs(a[k]));
    int idx = lane;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_xor(v, off, 64);
      int oi = __shfl_xor(idx, off, 64);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = idx;
    const double piv = __shfl(a[k], p, 64);
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) {
      if (lane == 0) atomicOr(flag + einst[e], 1);
      return;
    }
    if (lane == p) {
      const double pinv = 1.0 / piv;
#pragma unroll
      for (int j = 0; j < BU; ++j) a[j] = (j == k) ? pinv : a[j] * pinv;
#pragma unroll
      for (int j = 0; j < BU; ++j) prow[j] = a[j];
      used = true;
      mystep = k;
      s_pk[k] = p;
    }
    __syncthreads();
    if (lane != p && lane < BU) {
      const double f = a[k];
#pragma unroll
      for (int j = 0; j < BU; ++j) a[j] = (j == k) ? -f * prow[k] : a[j] - f * prow[j];
    }
    __syncthreads();
  }
  if (lane < BU) {
    double *out = inv + e * BU * BU;
    float *out32 = inv32 ? inv32 + e * BU * BU : nullptr;
#pragma unroll
    for (int k = 0; k < BU; ++k) {
      const int64_t o = (int64_t)s_pk[k] * BU + mystep;
      out[o] = a[k];
      if (out32) out32[o] = (float)a[k];
    }
  }
}

hipError_t launch_blockinv(const KParams &kp, const double *A, double *inv, float *inv32,
                           int *flag, hipStream_t st) {
  const int64_t ne = kp.s.ne;
  if (!ne) return hipSuccess;
  switch (kp.s.bu) {
    case 6: hipLaunchKernelGGL(k_blockinv<6>, dim3((unsigned)ne), dim3(64), 0, st, ne, kp.m.blk_ptr, kp.einst, A, inv, inv32, flag); break;
    case 12: hipLaunchKernelGGL(k_blockinv<12>, dim3((unsigned)ne), dim3(64), 0, st, ne, kp.m.blk_ptr, kp.einst, A, inv, inv32, flag); break;
    case 30: hipLaunchKernelGGL(k_blockinv<30>, dim3((unsigned)ne), dim3(64), 0, st, ne, kp.m.blk_ptr, kp.einst, A, inv, inv32, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Schur pressure block S = D - C M_A^-1 B (dense n_p x n_p) and its inverse
// ---------------------------------------------------------------------------
constexpr int kMaxStrip = 32;  // strip entries per element (<= (dim+1) * face nodes)

// per strip element: Z = inv_e B_e (bs x ns), T_e = C_e Z (ns x ns)
__global__ __launch_bounds__(64) void k_schur_t(KParams kp, const double *__restrict__ inv,
                                                const double *__restrict__ Bs,
                                                const double *__restrict__ Cs,
                                                double *__restrict__ T) {
  const int64_t se = blockIdx.x;
  const int tid = threadIdx.x;
  const int BU = kp.s.bu;
  const int64_t e = kp.m.strip_elems[se];
  const int64_t s0 = kp.m.sp_ptr[e];
  const int ns = (int)(kp.m.sp_ptr[e + 1] - s0);
  __shared__ double Z[kMaxStrip][32];
  const double *ie = inv + e * BU * BU;
  for (int t = tid; t < ns * BU; t += 64) {
    const int k = t / BU, r = t % BU;
    double acc = 0.0;
    for (int c = 0; c < BU; ++c) acc += ie[c * BU + r] * Bs[(s0 + k) * BU + c];
    Z[k][r] = acc;
  }
  __syncthreads();
  double *Te = T + kp.m.t_ptr[se];
  for (int t = tid; t < ns * ns; t += 64) {
    const int rho = t / ns, c2 = t % ns;
    double acc = 0.0;
    for (int r = 0; r < BU; ++r) acc += Cs[(s0 + rho) * BU + r] * Z[c2][r];
    Te[t] = acc;
  }
}

// per pressure row: S_b[i][:] = D_b[i][:] - sum of the T blocks that touch row i
__global__ void k_schur_gather(KParams kp, const double *__restrict__ D,
                               const double *__restrict__ T, const int32_t *__restrict__ sp_se,
                               double *__restrict__ S) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= kp.s.n_p) return;
  const int b = kp.pinst[i];
  const int64_t p0 = kp.poff[b], nb = kp.poff[b + 1] - p0;
  double *Srow = S + kp.doff[b] + (i - p0) * nb;
  const double *Drow = D + kp.doff[b] + (i - p0) * nb;
  for (int64_t j = 0; j < nb; ++j) Srow[j] = Drow[j];
  for (int32_t c = kp.m.pc_ptr[i]; c < kp.m.pc_ptr[i + 1]; ++c) {
    const int32_t ent = kp.m.pc_ent[c];
    const int64_t e = kp.m.sp_elem[ent];
    const int64_t s0 = kp.m.sp_ptr[e];
    const int ns = (int)(kp.m.sp_ptr[e + 1] - s0);
    const int rho = (int)(ent - s0);
    const double *Te = T + kp.m.t_ptr[sp_se[ent]];
    for (int c2 = 0; c2 < ns; ++c2) Srow[kp.m.sp_pnode[s0 + c2] - p0] -= Te[rho * ns + c2];
  }
}

// dense Gauss-Jordan inverse with partial pivoting, one workgroup, in place
constexpr int kMaxDenseP = 4096;
__global__ __launch_bounds__(256) void k_dense_inv(const int32_t *__restrict__ poff,
                                                   const int64_t *__restrict__ doff,
                                                   double *__restrict__ Wall,
                                                   double *__restrict__ outall,
                                                   float *__restrict__ out32all, int *flag) {
  const int bi = blockIdx.x;
  const int64_t n = poff[bi + 1] - poff[bi];
  double *W = Wall + doff[bi];
  double *out = outall + doff[bi];
  float *out32 = out32all + doff[bi];
  __shared__ double colk[kMaxDenseP];
  __shared__ int perm[kMaxDenseP];
  __shared__ double sv[256];
  __shared__ int si[256];
  const int tid = threadIdx.x;
  for (int64_t k = 0; k < n; ++k) {
    double v = -1.0;
    int idx = (int)n;
    for (int64_t r = k + tid; r < n; r += 256) {
      double a = fabs(W[r * n + k]);
      if (a > v || (a == v && r < idx)) {
        v = a;
        idx = (int)r;
      }
    }
    sv[tid] = v;
    si[tid] = idx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        double ov = sv[tid + s];
        int oi = si[tid + s];
        if (ov > sv[tid] || (ov == sv[tid] && oi < si[tid])) {
          sv[tid] = ov;
          si[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int p = si[0];
    const double pv = (p < n) ? W[(int64_t)p * n + k] : 0.0;
    __syncthreads();
    if (!(fabs(pv) > 0.0) || !isfinite(pv)) {
      if (tid == 0) atomicOr(flag + bi, 2);
      return;
    }
    if (tid == 0) perm[k] = p;
    if (p != k)
      for (int64_t j = tid; j < n; j += 256) {
        double t = W[k * n + j];
        W[k * n + j] = W[(int64_t)p * n + j];
        W[(int64_t)p * n + j] = t;
      }
    __syncthreads();
    const double pinv = 1.0 / pv;
    for (int64_t j = tid; j < n; j += 256) W[k * n + j] = (j == k) ? pinv : W[k * n + j] * pinv;
    for (int64_t r = tid; r < n; r += 256) colk[r] = W[r * n + k];
    __syncthreads();
    for (int64_t t = tid; t < n * n; t += 256) {
      const int64_t r = t / n, j = t % n;
      if (r == k) continue;
      const double f = colk[r];
      W[t] = (j == k) ? -f * pinv : W[t] - f * W[k * n + j];
    }
    __syncthreads();
  }
  for (int64_t k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int64_t r = tid; r < n; r += 256) {
        double t = W[r * n + k];
        W[r * n + k] = W[r * n + p];
        W[r * n + p] = t;
      }
    __syncthreads();
  }
  for (int64_t t = tid; t < n * n; t += 256) {
    out[t] = W[t];
    out32[t] = (float)W[t];
  }
}

hipError_t launch_schur(const KParams &kp, const double *inv, const double *Bs,
                        const double *Cs, const double *D, double *Z, double *T, double *S,
                        double *Sinv, float *Sinv32, int *flag, hipStream_t st) {
  (void)Z;
  const int64_t np = kp.s.n_p;
  if (!np) return hipSuccess;
  if (kp.s.n_se)
    hipLaunchKernelGGL(k_schur_t, dim3((unsigned)kp.s.n_se), dim3(64), 0, st, kp, inv, Bs, Cs, T);
  hipLaunchKernelGGL(k_schur_gather, dim3((unsigned)((np + 63) / 64)), dim3(64), 0, st, kp, D, T,
                     kp.m.sp_se, S);
  hipLaunchKernelGGL(k_dense_inv, dim3(kp.n_inst), dim3(256), 0, st, kp.poff, kp.doff, S, Sinv,
                     Sinv32, flag);
  return hipGetLastError();
}

__global__ void k_convert(const double *__restrict__ in, float *__restrict__ out, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    out[t] = (float)in[t];
}
hipError_t launch_convert(const double *in, float *out, int64_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)g), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Krylov vector kernels.  Reductions: each block writes one partial per
// output in a fixed order; k_reduce sums the partials of each output in a
// fixed tree.  Results are therefore bitwise reproducible for a given size.
// ---------------------------------------------------------------------------
constexpr int kRedThreads = 256;
constexpr int kMaxBlocks = 1024;

int reduce_blocks(int64_t n) {
  int64_t b = (n + 2047) / 2048;
  if (b < 1) b = 1;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return (int)b;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// block partial of k dot products (or norms) -> partial[blockIdx*k + i]
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_mdot(const T *__restrict__ V, int64_t ldv, int k,
                                                      const T *__restrict__ w, int64_t n,
                                                      double *__restrict__ partial) {
  __shared__ double wsum[kMaxKrylov][kRedThreads / 64];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  for (int i = 0; i < k; ++i) {
    double acc = 0.0;
    const T *vi = V + i * ldv;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kRedThreads) acc += (double)vi[r] * (double)w[r];
    acc = wave_sum(acc);
    if (lane == 0) wsum[i][wv] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kRedThreads) {
    double s = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) s += wsum[i][q];
    partial[(int64_t)blockIdx.x * k + i] = s;
  }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const double *__restrict__ partial, int nblk,
                                                        int k, double *__restrict__ out) {
  __shared__ double sm[kRedThreads];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kRedThreads) acc += partial[(int64_t)b * k + i];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = sm[0];
}

hipError_t launch_reduce_partials(const double *partial, int nblk, int k, double *out,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kRedThreads), 0, st, partial, nblk, k, out);
  return hipGetLastError();
}

__global__ void k_fill(double v, double *__restrict__ x, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    x[t] = v;
}
hipError_t launch_fill(double v, double *x, int64_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)g), dim3(256), 0, st, v, x, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mdot(const T *V, int64_t ldv, int k, const T *w, int64_t n, double *partial,
                       double *out, hipStream_t st) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL(k_mdot<T>, dim3(nb), dim3(kRedThreads), 0, st, V, ldv, k, w, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kRedThreads), 0, st, partial, nb, k, out);
  return hipGetLastError();
}
template hipError_t launch_mdot<double>(const double *, int64_t, int, const double *, int64_t,
                                        double *, double *, hipStream_t);
template hipError_t launch_mdot<float>(const float *, int64_t, int, const float *, int64_t,
                                       double *, double *, hipStream_t);

// w -= sum_i h_i V_i ; then partial dots V_i . w (MODE 1) or ||w||^2 (MODE 2)
template <typename T, int MODE>
__global__ __launch_bounds__(kRedThreads) void k_update(const T *__restrict__ V, int64_t ldv, int k,
                                                        const double *__restrict__ h,
                                                        T *__restrict__ w, int64_t n,
                                                        double *__restrict__ partial) {
  __shared__ double sh[kMaxKrylov];
  __shared__ double wsum[kMaxKrylov][kRedThreads / 64];
  for (int i = threadIdx.x; i < k; i += kRedThreads) sh[i] = h[i];
  __syncthreads();
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  double nacc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kRedThreads) {
    double acc = (double)w[r];
    for (int i = 0; i < k; ++i) acc -= sh[i] * (double)V[i * ldv + r];
    const T wr = (T)acc;
    w[r] = wr;
    nacc += (double)wr * (double)wr;
  }
  if (MODE == 2) {
    nacc = wave_sum(nacc);
    if (lane == 0) wsum[0][wv] = nacc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int q = 0; q < kRedThreads / 64; ++q) s += wsum[0][q];
      partial[blockIdx.x] = s;
    }
    return;
  }
  // MODE 1: partial dots with the updated w (re-read of this block's rows)
  __syncthreads();
  for (int i = 0; i < k; ++i) {
    double acc = 0.0;
    const T *vi = V + i * ldv;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += kRedThreads) acc += (double)vi[r] * (double)w[r];
    acc = wave_sum(acc);
    if (lane == 0) wsum[i][wv] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += kRedThreads) {
    double s = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) s += wsum[i][q];
    partial[(int64_t)blockIdx.x * k + i] = s;
  }
}

template <typename T>
hipError_t launch_update_mdot(const T *V, int64_t ldv, int k, const double *h, T *w, int64_t n,
                              double *partial, double *out, hipStream_t st) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL((k_update<T, 1>), dim3(nb), dim3(kRedThreads), 0, st, V, ldv, k, h, w, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(k), dim3(kRedThreads), 0, st, partial, nb, k, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_update_norm(const T *V, int64_t ldv, int k, const double *h, T *w, int64_t n,
                              double *partial, double *out, hipStream_t st) {
  const int nb = reduce_blocks(n);
  hipLaunchKernelGGL((k_update<T, 2>), dim3(nb), dim3(kRedThreads), 0, st, V, ldv, k, h, w, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, st, partial, nb, 1, out);
  return hipGetLastError();
}
template hipError_t launch_update_mdot<double>(const double *, int64_t, int, const double *,
                                               double *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_update_mdot<float>(const float *, int64_t, int, const double *,
                                              float *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_update_norm<double>(const double *, int64_t, int, const double *,
                                               double *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_update_norm<float>(const float *, int64_t, int, const double *,
                                              float *, int64_t, double *, double *, hipStream_t);

// ---------------------------------------------------------------------------
// Gram-Schmidt passes with register tiling.  A block owns OR_ROWS rows per
// thread (1024 rows); w stays in registers while the basis vectors stream in
// tiles of OR_TILE, so every thread keeps OR_ROWS * OR_TILE loads in flight.
// ---------------------------------------------------------------------------
constexpr int OR_ROWS = 4;
constexpr int OR_TILE = 8;
constexpr int OR_CHUNK = kRedThreads * OR_ROWS;

int ortho_blocks(int64_t n) { return (int)((n + OR_CHUNK - 1) / OR_CHUNK); }

// partial[b*(k+1) + i] = sum over the block's rows of V_i w (i < k), and
// partial[b*(k+1) + k] = sum of w^2
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_proj(const T *__restrict__ V, int64_t ldv, int k,
                                                      const T *__restrict__ w, int64_t n,
                                                      double *__restrict__ partial) {
  __shared__ double wsum[kMaxKrylov + 1][kRedThreads / 64];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t r0 = (int64_t)blockIdx.x * OR_CHUNK + tid;
  double wr[OR_ROWS];
  double nn = 0.0;
#pragma unroll
  for (int s = 0; s < OR_ROWS; ++s) {
    const int64_t r = r0 + (int64_t)s * kRedThreads;
    wr[s] = r < n ? (double)w[r] : 0.0;
    nn += wr[s] * wr[s];
  }
  for (int i0 = 0; i0 < k; i0 += OR_TILE) {
    double acc[OR_TILE];
#pragma unroll
    for (int q = 0; q < OR_TILE; ++q) acc[q] = 0.0;
#pragma unroll
    for (int s = 0; s < OR_ROWS; ++s) {
      const int64_t r = r0 + (int64_t)s * kRedThreads;
      if (r < n) {
#pragma unroll
        for (int q = 0; q < OR_TILE; ++q)
          if (i0 + q < k) acc[q] += (double)V[(int64_t)(i0 + q) * ldv + r] * wr[s];
      }
    }
#pragma unroll
    for (int q = 0; q < OR_TILE; ++q) {
      const double v = wave_sum(acc[q]);
      if (lane == 0 && i0 + q < k) wsum[i0 + q][wv] = v;
    }
  }
  nn = wave_sum(nn);
  if (lane == 0) wsum[k][wv] = nn;
  __syncthreads();
  for (int i = tid; i <= k; i += kRedThreads) {
    double s2 = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) s2 += wsum[i][q];
    partial[(int64_t)blockIdx.x * (k + 1) + i] = s2;
  }
}

// w -= sum_i h_i V_i ; partial[b] = sum of the new w^2
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_orth_update(const T *__restrict__ V, int64_t ldv,
                                                             int k, const double *__restrict__ h,
                                                             T *__restrict__ w, int64_t n,
                                                             double *__restrict__ partial) {
  __shared__ double sh[kMaxKrylov];
  __shared__ double wsum[kRedThreads / 64];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  for (int i = tid; i < k; i += kRedThreads) sh[i] = h[i];
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * OR_CHUNK + tid;
  double acc[OR_ROWS];
#pragma unroll
  for (int s = 0; s < OR_ROWS; ++s) {
    const int64_t r = r0 + (int64_t)s * kRedThreads;
    acc[s] = r < n ? (double)w[r] : 0.0;
  }
  for (int i0 = 0; i0 < k; i0 += OR_TILE) {
#pragma unroll
    for (int s = 0; s < OR_ROWS; ++s) {
      const int64_t r = r0 + (int64_t)s * kRedThreads;
      if (r < n) {
#pragma unroll
        for (int q = 0; q < OR_TILE; ++q)
          if (i0 + q < k) acc[s] -= sh[i0 + q] * (double)V[(int64_t)(i0 + q) * ldv + r];
      }
    }
  }
  double nn = 0.0;
#pragma unroll
  for (int s = 0; s < OR_ROWS; ++s) {
    const int64_t r = r0 + (int64_t)s * kRedThreads;
    if (r < n) {
      const T v = (T)acc[s];
      w[r] = v;
      nn += (double)v * (double)v;
    }
  }
  nn = wave_sum(nn);
  if (lane == 0) wsum[wv] = nn;
  __syncthreads();
  if (tid == 0) {
    double s2 = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) s2 += wsum[q];
    partial[blockIdx.x] = s2;
  }
}

template <typename T>
hipError_t launch_proj(const T *V, int64_t ldv, int k, const T *w, int64_t n, double *partial,
                       double *out, hipStream_t st) {
  const int nb = ortho_blocks(n);
  hipLaunchKernelGGL(k_proj<T>, dim3(nb), dim3(kRedThreads), 0, st, V, ldv, k, w, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(k + 1), dim3(kRedThreads), 0, st, partial, nb, k + 1, out);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_orth_update(const T *V, int64_t ldv, int k, const double *h, T *w, int64_t n,
                              double *partial, double *out, hipStream_t st) {
  const int nb = ortho_blocks(n);
  hipLaunchKernelGGL(k_orth_update<T>, dim3(nb), dim3(kRedThreads), 0, st, V, ldv, k, h, w, n, partial);
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, st, partial, nb, 1, out);
  return hipGetLastError();
}
template hipError_t launch_proj<double>(const double *, int64_t, int, const double *, int64_t,
                                        double *, double *, hipStream_t);
template hipError_t launch_proj<float>(const float *, int64_t, int, const float *, int64_t,
                                       double *, double *, hipStream_t);
template hipError_t launch_orth_update<double>(const double *, int64_t, int, const double *,
                                               double *, int64_t, double *, double *, hipStream_t);
template hipError_t launch_orth_update<float>(const float *, int64_t, int, const double *,
                                              float *, int64_t, double *, double *, hipStream_t);

static inline dim3 grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}
#define GRID_STRIDE(t, n) \
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (n); t += (int64_t)gridDim.x * blockDim.x)

template <typename T>
__global__ void k_scale_copy(const T *__restrict__ w, double s, T *__restrict__ v, int64_t n) {
  GRID_STRIDE(t, n) v[t] = (T)((double)w[t] * s);
}
template <typename T>
hipError_t launch_scale_copy(const T *w, double inv_norm, T *v, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy<T>, grid_for(n), dim3(256), 0, st, w, inv_norm, v, n);
  return hipGetLastError();
}
template hipError_t launch_scale_copy<double>(const double *, double, double *, int64_t, hipStream_t);
template hipError_t launch_scale_copy<float>(const float *, double, float *, int64_t, hipStream_t);

template <typename T>
__global__ void k_combine(const T *__restrict__ V, int64_t ldv, int k, const double *__restrict__ y,
                          T *__restrict__ out, int64_t n) {
  __shared__ double sy[kMaxKrylov];
  for (int i = threadIdx.x; i < k; i += blockDim.x) sy[i] = y[i];
  __syncthreads();
  GRID_STRIDE(t, n) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += sy[i] * (double)V[i * ldv + t];
    out[t] = (T)acc;
  }
}
template <typename T>
hipError_t launch_combine(const T *V, int64_t ldv, int k, const double *y, T *out, int64_t n,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_combine<T>, grid_for(n), dim3(256), 0, st, V, ldv, k, y, out, n);
  return hipGetLastError();
}
template hipError_t launch_combine<double>(const double *, int64_t, int, const double *, double *,
                                           int64_t, hipStream_t);
template hipError_t launch_combine<float>(const float *, int64_t, int, const double *, float *,
                                          int64_t, hipStream_t);

// y = a x + b y; a term with a zero coefficient is not read, so y may start
// uninitialised when b = 0
__global__ void k_axpby(double a, const double *__restrict__ x, double b, double *__restrict__ y,
                        int64_t n) {
  GRID_STRIDE(t, n) {
    double v = a == 0.0 ? 0.0 : a * x[t];
    if (b != 0.0) v += b * y[t];
    y[t] = v;
  }
}
hipError_t launch_axpby(double a, const double *x, double b, double *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, grid_for(n), dim3(256), 0, st, a, x, b, y, n);
  return hipGetLastError();
}
__global__ void k_cast_axpy(double a, const float *__restrict__ x, double *__restrict__ y, int64_t n) {
  GRID_STRIDE(t, n) y[t] += a * (double)x[t];
}
hipError_t launch_cast_axpy(double a, const float *x, double *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_axpy, grid_for(n), dim3(256), 0, st, a, x, y, n);
  return hipGetLastError();
}
__global__ void k_cast_scale(const double *__restrict__ x, double a, float *__restrict__ y, int64_t n) {
  GRID_STRIDE(t, n) y[t] = (float)(a * x[t]);
}
hipError_t launch_cast_scale(const double *x, double a, float *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_cast_scale, grid_for(n), dim3(256), 0, st, x, a, y, n);
  return hipGetLastError();
}
__global__ void k_sub(const double *__restrict__ b, const double *__restrict__ Jx,
                      double *__restrict__ r, int64_t n) {
  GRID_STRIDE(t, n) r[t] = b[t] - Jx[t];
}
hipError_t launch_sub(const double *b, const double *Jx, double *r, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_sub, grid_for(n), dim3(256), 0, st, b, Jx, r, n);
  return hipGetLastError();
}
template <typename T>
__global__ void k_sub_t(const T *__restrict__ b, const T *__restrict__ Jx, T *__restrict__ r,
                        int64_t n) {
  GRID_STRIDE(t, n) r[t] = b[t] - Jx[t];
}
template <typename T>
hipError_t launch_sub_t(const T *b, const T *Jx, T *r, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_sub_t<T>, grid_for(n), dim3(256), 0, st, b, Jx, r, n);
  return hipGetLastError();
}
template hipError_t launch_sub_t<double>(const double *, const double *, double *, int64_t, hipStream_t);
template hipError_t launch_sub_t<float>(const float *, const float *, float *, int64_t, hipStream_t);
template <typename T>
__global__ void k_axpy_t(double a, const T *__restrict__ x, T *__restrict__ y, int64_t n) {
  GRID_STRIDE(t, n) y[t] = (T)((double)y[t] + a * (double)x[t]);
}
template <typename T>
hipError_t launch_axpy_t(double a, const T *x, T *y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy_t<T>, grid_for(n), dim3(256), 0, st, a, x, y, n);
  return hipGetLastError();
}
template hipError_t launch_axpy_t<double>(double, const double *, double *, int64_t, hipStream_t);
template hipError_t launch_axpy_t<float>(double, const float *, float *, int64_t, hipStream_t);

// u += du, p += dp (optional cut-off); partials of ||du||^2, ||u||^2, ||dp||^2, ||p||^2
__global__ __launch_bounds__(kRedThreads) void k_newton_update(const double *__restrict__ dx,
                                                               double *__restrict__ u, int64_t n_u,
                                                               double *__restrict__ p, int64_t n_p,
                                                               int cutoff_on, double cutoff,
                                                               double *__restrict__ partial) {
  __shared__ double wsum[4][kRedThreads / 64];
  const int64_t n = n_u + n_p;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = blockIdx.x * chunk, r1 = min(n, r0 + chunk);
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kRedThreads) {
    const double d = dx[r];
    if (r < n_u) {
      const double v = u[r] + d;
      u[r] = v;
      a[0] += d * d;
      a[1] += v * v;
    } else {
      double v = p[r - n_u] + d;
      if (cutoff_on && v < cutoff) v = cutoff;
      p[r - n_u] = v;
      a[2] += d * d;
      a[3] += v * v;
    }
  }
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  for (int c = 0; c < 4; ++c) {
    double s = wave_sum(a[c]);
    if (lane == 0) wsum[c][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) s += wsum[threadIdx.x][q];
    partial[(int64_t)blockIdx.x * 4 + threadIdx.x] = s;
  }
}
hipError_t launch_newton_update(const double *dx, double *u, int64_t n_u, double *p, int64_t n_p,
                                int cutoff_on, double cutoff, double *partial, double *out,
                                hipStream_t st) {
  const int nb = reduce_blocks(n_u + n_p);
  hipLaunchKernelGGL(k_newton_update, dim3(nb), dim3(kRedThreads), 0, st, dx, u, n_u, p, n_p,
                     cutoff_on, cutoff, partial);
  hipLaunchKernelGGL(k_reduce, dim3(4), dim3(kRedThreads), 0, st, partial, nb, 4, out);
  return hipGetLastError();
}

hipError_t launch_norm2(const double *x, int64_t n, double *partial, double *out, hipStream_t st) {
  return launch_mdot<double>(x, 0, 1, x, n, partial, out, st);
}

}  // namespace hf
