// Linear-algebra kernels for gfx950: batched inverses of the element
// blocks, the Schur pressure block and its inverse, precision conversion and
// vector fills.
#include <algorithm>
#include <cmath>

#include "hf_internal.h"

namespace hf {

// ---------------------------------------------------------------------------
// Batched inverse of the diagonal element blocks: Gauss-Jordan with partial
// (row) pivoting, one wavefront per block, lane r holds row r in registers.
// Pivot rows are chosen in place (no physical swap); the inverse is read out
// with the column permutation the pivot order implies.  A block is singular
// to working precision when a pivot is not larger than kSingularRel times its
// largest entry (the rounding residue of an exactly rank-deficient block,
// such as the stiffness of an element held by no face and no boundary
// condition, is a few units of 1e-16 of it), or when a pivot is not finite.
// ---------------------------------------------------------------------------
constexpr double kSingularRel = 1e-13;

template <int BU>
__global__ __launch_bounds__(64) void k_blockinv(const int32_t *__restrict__ elist,
                                                 const int64_t *__restrict__ blk_ptr,
                                                 const int32_t *__restrict__ einst,
                                                 const double *__restrict__ A,
                                                 double *__restrict__ inv,
                                                 float *__restrict__ inv32, int *flag) {
  const int64_t e = elist ? elist[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x;
  __shared__ double prow[BU];
  __shared__ int s_pk[BU];
  const double *blk = A + blk_ptr[e] * BU * BU;
  double a[BU];
#pragma unroll
  for (int c = 0; c < BU; ++c) a[c] = lane < BU ? blk[c * BU + lane] : 0.0;
  bool used = lane >= BU;
  int mystep = 0;
  double amax = 0.0;
#pragma unroll
  for (int c = 0; c < BU; ++c) amax = fmax(amax, isnan(a[c]) ? INFINITY : fabs(a[c]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, 64));
  const double tiny = kSingularRel * amax;
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
    if (!(fabs(piv) > tiny) || !isfinite(piv) || !isfinite(amax)) {
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
                           const int32_t *elist, int64_t n, int *flag, hipStream_t st) {
  if (!n) return hipSuccess;
  const dim3 g((unsigned)n), b(64);
  switch (kp.s.bu) {
    case 6: hipLaunchKernelGGL(k_blockinv<6>, g, b, 0, st, elist, kp.m.blk_ptr, kp.einst, A, inv, inv32, flag); break;
    case 12: hipLaunchKernelGGL(k_blockinv<12>, g, b, 0, st, elist, kp.m.blk_ptr, kp.einst, A, inv, inv32, flag); break;
    case 30: hipLaunchKernelGGL(k_blockinv<30>, g, b, 0, st, elist, kp.m.blk_ptr, kp.einst, A, inv, inv32, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 inverses of the 30 x 30 element blocks on the matrix cores.  A block
// is padded to 32 x 32 (identity in the padding) and split into 16 x 16
// tiles [[A11, A12], [A21, A22]]:
//   X = A11^-1, T = A21 X, S = A22 - T A12, Y = S^-1, U = X A12,
//   inverse = [[X + U Y T, -U Y], [-Y T, Y]].
// The two 16 x 16 inverses are Gauss-Jordan with partial pivoting inside the
// tile; the six 16 x 16 x 16 products are v_mfma_f32_16x16x4f32 chains
// (4 per product).  One wavefront per block, all tiles in LDS.  A zero or
// non-finite pivot in a tile (possible even for an invertible block, since
// pivoting does not cross tiles) sets flag bit 4 for the block's instance;
// the caller then falls back to the FP64 Gauss-Jordan inverses.
// ---------------------------------------------------------------------------
typedef float floatx4 __attribute__((ext_vector_type(4)));

// c += a b for 16 x 16 tiles in LDS (row-major, leading dimensions la, lb).
// Operand layout of the 16x16x4 instruction: lane l supplies a[l%16][4q + l/16]
// and b[4q + l/16][l%16]; the accumulator's register r of lane l is
// c[4(l/16) + r][l%16].
__device__ inline floatx4 mfma16(const float *a, int la, const float *b, int lb, floatx4 c, int lane) {
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i * la + 4 * q + kq], b[(4 * q + kq) * lb + i], c, 0, 0, 0);
  return c;
}
__device__ inline floatx4 tile_load(const float *t, int ld, int lane) {
  const int j = lane & 15, i0 = 4 * (lane >> 4);
  floatx4 v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = t[(i0 + r) * ld + j];
  return v;
}
__device__ inline void tile_store(float *t, int ld, floatx4 v, int lane) {
  const int j = lane & 15, i0 = 4 * (lane >> 4);
#pragma unroll
  for (int r = 0; r < 4; ++r) t[(i0 + r) * ld + j] = v[r];
}

// in-place Gauss-Jordan inverse of a 16 x 16 LDS tile with partial pivoting
// (row swaps, undone on the columns at the end); false on a zero or
// non-finite pivot (uniform over the wavefront)
__device__ bool gj16(float *M, int ld, int *perm, int lane) {
  for (int k = 0; k < 16; ++k) {
    float v = -1.f;
    int idx = 16;
    if (lane >= k && lane < 16) {
      const float a = fabsf(M[lane * ld + k]);
      v = isnan(a) ? INFINITY : a;  // NaN is picked and reported
      idx = lane;
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) {
      const float ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(idx, off, 64);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = __shfl(idx, 0, 64);
    const float piv = M[p * ld + k];
    if (!(fabsf(piv) > 0.f) || !isfinite(piv)) return false;
    if (p != k && lane < 16) {
      const float t = M[k * ld + lane];
      M[k * ld + lane] = M[p * ld + lane];
      M[p * ld + lane] = t;
    }
    if (lane == 0) perm[k] = p;
    __syncthreads();
    const float pinv = 1.f / piv;
    if (lane < 16) M[k * ld + lane] = lane == k ? pinv : M[k * ld + lane] * pinv;
    __syncthreads();
    float f[4], rk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = lane + 64 * q, r = t >> 4, c = t & 15;
      f[q] = M[r * ld + k];
      rk[q] = M[k * ld + c];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = lane + 64 * q, r = t >> 4, c = t & 15;
      if (r != k) M[r * ld + c] = c == k ? -f[q] * pinv : M[r * ld + c] - f[q] * rk[q];
    }
    __syncthreads();
  }
  for (int k = 15; k >= 0; --k) {
    const int p = perm[k];
    if (p != k && lane < 16) {
      const float t = M[lane * ld + k];
      M[lane * ld + k] = M[lane * ld + p];
      M[lane * ld + p] = t;
    }
    __syncthreads();
  }
  return true;
}

__global__ __launch_bounds__(64) void k_blockinv32_mfma(const int32_t *__restrict__ elist,
                                                        const int64_t *__restrict__ blk_ptr,
                                                        const int32_t *__restrict__ einst,
                                                        const double *__restrict__ A,
                                                        float *__restrict__ inv32, int *flag) {
  constexpr int BU = 30, LD = 33, LT = 17;
  __shared__ float M[32 * LD];
  __shared__ float T[16 * LT], W[16 * LT];
  __shared__ int perm[16];
  const int64_t e = elist ? elist[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x;
  const double *blk = A + blk_ptr[e] * BU * BU;
  for (int t = lane; t < 32 * 32; t += 64) {
    const int r = t & 31, c = t >> 5;
    M[r * LD + c] = (r < BU && c < BU) ? (float)blk[c * BU + r] : (r == c ? 1.f : 0.f);
  }
  __syncthreads();
  float *A11 = M, *A12 = M + 16, *A21 = M + 16 * LD, *A22 = M + 16 * LD + 16;
  const floatx4 zero = {0.f, 0.f, 0.f, 0.f};
  bool ok = gj16(A11, LD, perm, lane);  // X
  if (ok) {
    tile_store(T, LT, mfma16(A21, LD, A11, LD, zero, lane), lane);  // T = A21 X
    __syncthreads();
    const floatx4 s = tile_load(A22, LD, lane) - mfma16(T, LT, A12, LD, zero, lane);
    __syncthreads();
    tile_store(A22, LD, s, lane);  // S
    __syncthreads();
    ok = gj16(A22, LD, perm, lane);  // Y
  }
  if (!ok) {
    if (lane == 0) atomicOr(flag + einst[e], 4);
    return;
  }
  tile_store(W, LT, mfma16(A11, LD, A12, LD, zero, lane), lane);  // U = X A12
  __syncthreads();
  const floatx4 b12 = -mfma16(W, LT, A22, LD, zero, lane);  // -U Y
  const floatx4 b21 = -mfma16(A22, LD, T, LT, zero, lane);  // -Y T
  __syncthreads();
  tile_store(A12, LD, b12, lane);
  tile_store(A21, LD, b21, lane);
  __syncthreads();
  const floatx4 b11 = tile_load(A11, LD, lane) - mfma16(A12, LD, T, LT, zero, lane);  // X + U Y T
  __syncthreads();
  tile_store(A11, LD, b11, lane);
  __syncthreads();
  float *out = inv32 + e * BU * BU;
  for (int t = lane; t < BU * BU; t += 64) {
    const int r = t % BU, c = t / BU;
    out[t] = M[r * LD + c];  // column-major, like the FP64 blocks
  }
}

hipError_t launch_blockinv32_mfma(const KParams &kp, const double *A, float *inv32,
                                  const int32_t *elist, int64_t n, int *flag, hipStream_t st) {
  if (kp.s.bu != 30) return hipErrorInvalidValue;
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_blockinv32_mfma, dim3((unsigned)n), dim3(64), 0, st, elist, kp.m.blk_ptr,
                     kp.einst, A, inv32, flag);
  return hipGetLastError();
}

// FP32 copies of the row panels of the listed elements
__global__ void k_convert_panels(const int32_t *__restrict__ elist, const int64_t *__restrict__ blk_ptr,
                                 int bs2, const double *__restrict__ A, float *__restrict__ A32) {
  const int64_t e = elist[blockIdx.x];
  const int64_t b0 = blk_ptr[e] * bs2, b1 = blk_ptr[e + 1] * bs2;
  for (int64_t t = b0 + threadIdx.x; t < b1; t += blockDim.x) A32[t] = (float)A[t];
}
hipError_t launch_convert_panels(const KParams &kp, const int32_t *elist, int64_t n, const double *A,
                                 float *A32, hipStream_t st) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_convert_panels, dim3((unsigned)n), dim3(256), 0, st, elist, kp.m.blk_ptr,
                     kp.s.bu * kp.s.bu, A, A32);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Folded right-preconditioned operator J M^-1: every block of the row panels
// times the inverse of its column element, Af_ef = A_ef inv_f, and every C
// strip entry times its element's inverse, Cf = C_e inv_e (the B strips and
// D are used with S^-1 x_p at product time).  FP64 arithmetic; TI is the
// precision of the inverses (FP64, or the FP32 set of GMRES-IR) and TO that
// of the result.
// ---------------------------------------------------------------------------
template <int BU, typename TI, typename TO>
__global__ __launch_bounds__(256) void k_fold_blocks(int64_t n_blocks, const int32_t *__restrict__ blist,
                                                     const int32_t *__restrict__ blk_col,
                                                     const double *__restrict__ A,
                                                     const TI *__restrict__ inv, TO *__restrict__ Af) {
  constexpr int B2 = BU * BU;
  __shared__ double sa[B2], si[B2];
  if ((int64_t)blockIdx.x >= n_blocks) return;
  const int64_t blk = blist ? (int64_t)blist[blockIdx.x] : (int64_t)blockIdx.x;
  const int64_t f = blk_col[blk];
  const double *a = A + blk * B2;
  const TI *iv = inv + f * B2;
  for (int t = threadIdx.x; t < B2; t += blockDim.x) {
    sa[t] = a[t];
    si[t] = (double)iv[t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < B2; t += blockDim.x) {  // column-major: t = r + c BU
    const int r = t % BU, c = t / BU;
    double acc = 0.0;
#pragma unroll 6
    for (int k = 0; k < BU; ++k) acc += sa[r + k * BU] * si[k + c * BU];
    Af[blk * B2 + t] = (TO)acc;
  }
}

template <int BU, typename TI, typename TO>
__global__ __launch_bounds__(256) void k_fold_cstrips(int64_t n_strip, const int32_t *__restrict__ sp_elem,
                                                      const double *__restrict__ Cs,
                                                      const TI *__restrict__ inv, TO *__restrict__ Cf) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n_strip * BU) return;
  const int64_t ent = t / BU;
  const int c = (int)(t % BU);
  const TI *iv = inv + (int64_t)sp_elem[ent] * BU * BU;
  double acc = 0.0;
  for (int r = 0; r < BU; ++r) acc += Cs[ent * BU + r] * (double)iv[r + c * BU];
  Cf[t] = (TO)acc;
}

template <int BU, typename TI, typename TO>
static void fold_bu(const KParams &kp, const double *A, const double *Cs, const TI *inv, TO *Af, TO *Cf,
                    const int32_t *blist, int64_t nblk, hipStream_t st) {
  constexpr int NT = BU * BU >= 256 ? 256 : (BU * BU + 63) / 64 * 64;
  if (nblk)
    hipLaunchKernelGGL((k_fold_blocks<BU, TI, TO>), dim3((unsigned)nblk), dim3(NT), 0, st, nblk, blist,
                       kp.m.blk_col, A, inv, Af);
  const int64_t nc = kp.s.n_strip * BU;
  if (nc)
    hipLaunchKernelGGL((k_fold_cstrips<BU, TI, TO>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st,
                       kp.s.n_strip, kp.m.sp_elem, Cs, inv, Cf);
}

template <typename TI, typename TO>
hipError_t launch_fold(const KParams &kp, const double *A, const double *Cs, const TI *inv, TO *Af, TO *Cf,
                       const int32_t *blist, int64_t nblk, hipStream_t st) {
  if (!blist) nblk = kp.s.n_blocks;
  switch (kp.s.bu) {
    case 6: fold_bu<6>(kp, A, Cs, inv, Af, Cf, blist, nblk, st); break;
    case 12: fold_bu<12>(kp, A, Cs, inv, Af, Cf, blist, nblk, st); break;
    case 30: fold_bu<30>(kp, A, Cs, inv, Af, Cf, blist, nblk, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_fold<double, double>(const KParams &, const double *, const double *,
                                                const double *, double *, double *, const int32_t *, int64_t,
                                                hipStream_t);
template hipError_t launch_fold<float, float>(const KParams &, const double *, const double *, const float *,
                                              float *, float *, const int32_t *, int64_t, hipStream_t);

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

// dense Gauss-Jordan inverse with partial pivoting, one workgroup of 1024
// threads per instance, in place; the elimination runs over a 32 x 32 thread
// grid (rows by ty, columns by tx)
constexpr int kMaxDenseP = 4096;
constexpr int kDT = 1024;
__global__ __launch_bounds__(kDT) void k_dense_inv(const int32_t *__restrict__ poff,
                                                   const int64_t *__restrict__ doff,
                                                   double *__restrict__ Wall,
                                                   double *__restrict__ outall,
                                                   float *__restrict__ out32all, int *flag, int n_wide) {
  const int bi = blockIdx.x;
  const int n = poff[bi + 1] - poff[bi];
  if (n_wide > 0 && n >= n_wide) return;  // left to the grid-wide steps below
  double *W = Wall + doff[bi];
  double *out = outall + doff[bi];
  float *out32 = out32all + doff[bi];
  __shared__ double colk[kMaxDenseP];
  __shared__ int perm[kMaxDenseP];
  __shared__ double sv[kDT];
  __shared__ int si[kDT];
  const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
  for (int k = 0; k < n; ++k) {
    double v = -1.0;
    int idx = n;
    for (int r = k + tid; r < n; r += kDT) {
      const double a = fabs(W[(int64_t)r * n + k]);
      if (a > v || (a == v && r < idx)) {
        v = a;
        idx = r;
      }
    }
    sv[tid] = v;
    si[tid] = idx;
    __syncthreads();
    for (int s2 = kDT / 2; s2 > 0; s2 >>= 1) {
      if (tid < s2) {
        const double ov = sv[tid + s2];
        const int oi = si[tid + s2];
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
      for (int j = tid; j < n; j += kDT) {
        const double t = W[(int64_t)k * n + j];
        W[(int64_t)k * n + j] = W[(int64_t)p * n + j];
        W[(int64_t)p * n + j] = t;
      }
    __syncthreads();
    const double pinv = 1.0 / pv;
    for (int j = tid; j < n; j += kDT) W[(int64_t)k * n + j] = (j == k) ? pinv : W[(int64_t)k * n + j] * pinv;
    for (int r = tid; r < n; r += kDT) colk[r] = W[(int64_t)r * n + k];
    __syncthreads();
    const double *Wk = W + (int64_t)k * n;
    for (int r = ty; r < n; r += kDT / 32) {
      if (r == k) continue;
      const double f = colk[r];
      double *Wr = W + (int64_t)r * n;
      for (int j = tx; j < n; j += 32) Wr[j] = (j == k) ? -f * pinv : Wr[j] - f * Wk[j];
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int r = tid; r < n; r += kDT) {
        const double t = W[(int64_t)r * n + k];
        W[(int64_t)r * n + k] = W[(int64_t)r * n + p];
        W[(int64_t)r * n + p] = t;
      }
    __syncthreads();
  }
  for (int64_t t = tid; t < (int64_t)n * n; t += kDT) {
    out[t] = W[t];
    out32[t] = (float)W[t];
  }
}

// The same Gauss-Jordan with partial pivoting for one large pressure block,
// blocked over panels of kGjPanel pivots so that the matrix is swept once per
// panel instead of once per pivot.  A pivot step k of the unblocked form
// exchanges whole rows k and p, scales row k by 1/W_kk and subtracts f_r times
// row k from every other row r (f_r = W_rk), storing -f_r/W_kk and 1/W_kk in
// column k.  For a panel K = [k0, k1) those steps act on a column j outside
// K as x <- P x, then x <- x + (W[:, K] - I[:, K]) x[K] with the panel
// columns as they stand after the panel (P: the panel's row exchanges, which
// the pivot kernel applies to whole rows at once).  So each panel runs its
// pivot steps on its own columns (k_gjb_pivot, k_gjb_panel), stages the pivot
// rows (k_gjb_stage) and updates every other column with one rank-|K|
// product (k_gjb_update); at the end the row exchanges are undone on the
// columns, last to first, as one gather (k_gjb_perm, k_gjb_finish).
__global__ __launch_bounds__(kDT) void k_gjb_pivot(double *__restrict__ W, int n, int k, int k0, int k1,
                                                   double *__restrict__ colk, int *__restrict__ perm,
                                                   double *__restrict__ piv, int *__restrict__ flag) {
  __shared__ double sv[kDT];
  __shared__ int si[kDT];
  const int tid = threadIdx.x;
  if (*flag & 2) {  // an earlier pivot failed: nothing more to do
    if (tid == 0) piv[0] = 0.0;
    return;
  }
  double v = -1.0;
  int idx = n;
  for (int r = k + tid; r < n; r += kDT) {
    const double a = fabs(W[(int64_t)r * n + k]);
    if (a > v || (a == v && r < idx)) {
      v = a;
      idx = r;
    }
  }
  sv[tid] = v;
  si[tid] = idx;
  __syncthreads();
  for (int s2 = kDT / 2; s2 > 0; s2 >>= 1) {
    if (tid < s2) {
      const double ov = sv[tid + s2];
      const int oi = si[tid + s2];
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
    if (tid == 0) {
      atomicOr(flag, 2);
      piv[0] = 0.0;
    }
    return;
  }
  if (tid == 0) perm[k] = p;
  if (p != k)
    for (int j = tid; j < n; j += kDT) {
      const double t = W[(int64_t)k * n + j];
      W[(int64_t)k * n + j] = W[(int64_t)p * n + j];
      W[(int64_t)p * n + j] = t;
    }
  __syncthreads();
  const double pinv = 1.0 / pv;
  for (int j = k0 + tid; j < k1; j += kDT) W[(int64_t)k * n + j] = (j == k) ? pinv : W[(int64_t)k * n + j] * pinv;
  __syncthreads();
  for (int r = tid; r < n; r += kDT) colk[r] = W[(int64_t)r * n + k];
  if (tid == 0) piv[0] = pinv;
}

// the panel columns of every row but k: W_rj -= f_r W_kj, and column k
// becomes -f_r / W_kk
__global__ __launch_bounds__(256) void k_gjb_panel(double *__restrict__ W, int n, int k, int k0, int k1,
                                                   const double *__restrict__ colk,
                                                   const double *__restrict__ piv) {
  const double pinv = piv[0];
  if (pinv == 0.0) return;  // failed pivot
  const int w = k1 - k0;
  const double *Wk = W + (int64_t)k * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * w;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / w), j = k0 + (int)(t % w);
    if (r == k) continue;
    const double f = colk[r];
    W[(int64_t)r * n + j] = (j == k) ? -f * pinv : W[(int64_t)r * n + j] - f * Wk[j];
  }
}

// X[i][j] = W[k0 + i][j]: the panel's pivot rows after the exchanges
__global__ __launch_bounds__(256) void k_gjb_stage(const double *__restrict__ W, int n, int k0, int k1,
                                                   double *__restrict__ X, const int *__restrict__ flag) {
  if (*flag & 2) return;
  const int64_t m = (int64_t)(k1 - k0) * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < m; t += (int64_t)gridDim.x * blockDim.x)
    X[t] = W[(int64_t)k0 * n + t];
}

// every column j outside the panel: W_rj = [r outside K] W_rj + sum_i W_r,k0+i X_ij,
// on 64 x 64 tiles (4 x 4 per thread), the panel columns and pivot rows in LDS
constexpr int kGjTile = 64;
__global__ __launch_bounds__(256) void k_gjb_update(double *__restrict__ W, int n, int k0, int k1,
                                                    const double *__restrict__ X, const int *__restrict__ flag) {
  __shared__ double Pt[kGjTile][kGjPanel + 1];
  __shared__ double Xt[kGjPanel][kGjTile];
  if (*flag & 2) return;
  const int w = k1 - k0;
  const int r0 = blockIdx.y * kGjTile, c0 = blockIdx.x * kGjTile;
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  for (int t = tid; t < kGjTile * kGjPanel; t += 256) {
    const int rr = t / kGjPanel, i = t % kGjPanel;
    const int row = r0 + rr;
    Pt[rr][i] = (i < w && row < n) ? W[(int64_t)row * n + k0 + i] : 0.0;
  }
  for (int t = tid; t < kGjPanel * kGjTile; t += 256) {
    const int i = t / kGjTile, cc = t % kGjTile;
    const int col = c0 + cc;
    Xt[i][cc] = (i < w && col < n) ? X[(int64_t)i * n + col] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int i = 0; i < w; ++i) {
    double pa[4], xb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) pa[a] = Pt[ty * 4 + a][i];
#pragma unroll
    for (int b = 0; b < 4; ++b) xb[b] = Xt[i][tx + 16 * b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += pa[a] * xb[b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = r0 + ty * 4 + a;
    if (row >= n) continue;
    const bool in_panel = row >= k0 && row < k1;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int col = c0 + tx + 16 * b;
      if (col >= n || (col >= k0 && col < k1)) continue;
      double *e = W + (int64_t)row * n + col;
      *e = (in_panel ? 0.0 : *e) + acc[a][b];
    }
  }
}

// the column permutation that undoes the row exchanges, last to first:
// column c of the inverse is column idx[c] of W (one workgroup, in LDS)
static_assert(kMaxPressureBlock <= 65536, "pivot rows are staged as 16-bit indices");
__global__ __launch_bounds__(kDT) void k_gjb_perm(int n, const int *__restrict__ perm, int *__restrict__ idx,
                                                  const int *__restrict__ flag) {
  __shared__ uint16_t sp[kMaxPressureBlock], sx[kMaxPressureBlock];  // 64 KB at 16,384 nodes
  if (*flag & 2) return;
  for (int c = threadIdx.x; c < n; c += kDT) {
    sp[c] = (uint16_t)perm[c];
    sx[c] = (uint16_t)c;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = n - 1; k >= 0; --k) {
      const int p = sp[k];
      if (p != k) {
        const uint16_t t = sx[k];
        sx[k] = sx[p];
        sx[p] = t;
      }
    }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += kDT) idx[c] = sx[c];
}

__global__ __launch_bounds__(256) void k_gjb_finish(const double *__restrict__ W, int n, const int *__restrict__ idx,
                                                    double *__restrict__ out, float *__restrict__ out32,
                                                    const int *__restrict__ flag) {
  if (*flag & 2) return;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (int64_t)n * n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(t / n), c = (int)(t % n);
    const double v = W[(int64_t)r * n + idx[c]];
    out[t] = v;
    out32[t] = (float)v;
  }
}

hipError_t launch_dense_inv_wide(double *W, double *out, float *out32, int n, int *flag, double *colk, int *perm,
                                 double *piv, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > kMaxPressureBlock) return hipErrorInvalidValue;
  // scratch: colk holds n multipliers then the staged pivot rows (kGjPanel x n),
  // perm holds n pivot rows then the final column gather (n)
  double *X = colk + kMaxPressureBlock;
  int *idx = perm + kMaxPressureBlock;
  const int64_t nn = (int64_t)n * n;
  const unsigned gf = (unsigned)std::min<int64_t>((nn + 255) / 256, 4096);
  const int nt = (n + kGjTile - 1) / kGjTile;
  for (int k0 = 0; k0 < n; k0 += kGjPanel) {
    const int k1 = std::min(k0 + kGjPanel, n);
    const unsigned gp = (unsigned)std::min<int64_t>(((int64_t)n * (k1 - k0) + 255) / 256, 4096);
    for (int k = k0; k < k1; ++k) {
      hipLaunchKernelGGL(k_gjb_pivot, dim3(1), dim3(kDT), 0, st, W, n, k, k0, k1, colk, perm, piv, flag);
      hipLaunchKernelGGL(k_gjb_panel, dim3(gp), dim3(256), 0, st, W, n, k, k0, k1, colk, piv);
    }
    if (k1 - k0 < n) {  // columns outside the panel exist
      hipLaunchKernelGGL(k_gjb_stage, dim3(gp), dim3(256), 0, st, W, n, k0, k1, X, flag);
      hipLaunchKernelGGL(k_gjb_update, dim3(nt, nt), dim3(256), 0, st, W, n, k0, k1, X, flag);
    }
  }
  hipLaunchKernelGGL(k_gjb_perm, dim3(1), dim3(kDT), 0, st, n, perm, idx, flag);
  hipLaunchKernelGGL(k_gjb_finish, dim3(gf), dim3(256), 0, st, W, n, idx, out, out32, flag);
  return hipGetLastError();
}

hipError_t launch_schur_form(const KParams &kp, const double *inv, const double *Bs, const double *Cs,
                             const double *D, double *T, double *S, hipStream_t st) {
  const int64_t np = kp.s.n_p;
  if (!np) return hipSuccess;
  if (kp.s.n_se)
    hipLaunchKernelGGL(k_schur_t, dim3((unsigned)kp.s.n_se), dim3(64), 0, st, kp, inv, Bs, Cs, T);
  hipLaunchKernelGGL(k_schur_gather, dim3((unsigned)((np + 63) / 64)), dim3(64), 0, st, kp, D, T,
                     kp.m.sp_se, S);
  return hipGetLastError();
}

hipError_t launch_schur_invert(const KParams &kp, double *S, double *Sinv, float *Sinv32, int *flag, int n_wide,
                               hipStream_t st) {
  if (!kp.s.n_p) return hipSuccess;
  hipLaunchKernelGGL(k_dense_inv, dim3(kp.n_inst), dim3(kDT), 0, st, kp.poff, kp.doff, S, Sinv,
                     Sinv32, flag, n_wide);
  return hipGetLastError();
}

hipError_t launch_schur(const KParams &kp, const double *inv, const double *Bs,
                        const double *Cs, const double *D, double *Z, double *T, double *S,
                        double *Sinv, float *Sinv32, int *flag, int n_wide, hipStream_t st) {
  (void)Z;
  const hipError_t e = launch_schur_form(kp, inv, Bs, Cs, D, T, S, st);
  if (e != hipSuccess) return e;
  return launch_schur_invert(kp, S, Sinv, Sinv32, flag, n_wide, st);
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
// Vector fills and updates (the batched Krylov kernels are in hf_kernels_krylov.hip)
// ---------------------------------------------------------------------------
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

static inline dim3 grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}
#define GRID_STRIDE(t, n) \
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < (n); t += (int64_t)gridDim.x * blockDim.x)

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

}  // namespace hf
