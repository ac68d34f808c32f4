// Block-sparse Jacobian product and block-Jacobi apply for gfx950.
//
// Jacobian storage.  Element row e of A is one contiguous "row panel": its
// blocks (diagonal first, then one per interior face in local-face order)
// each stored column-major, so the panel is a column-major bs x (nb*bs)
// matrix.  The product streams each panel with 16-byte nontemporal loads: a
// group of L lanes reads CH = LA*EL consecutive values per step, and because
// CH is a multiple of bs every lane keeps the same rows at every step; the
// products are summed per lane and combined across lanes in a fixed order at
// the end.
// The x values a row panel needs are staged in LDS first.
#include <cmath>

#include <mutex>
#include <vector>

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

// lanes per element row: the wide shape (variant 0) or half of it (variant 1)
__host__ __device__ constexpr int wide_lanes(int BU) { return BU >= 24 ? 64 : (BU >= 12 ? 32 : 16); }

template <typename T, int BU, int L_>
struct SpmvShape {
  static constexpr int EL = Vec16<T>::EL;
  static constexpr int L = L_;
  static constexpr int LA = active_lanes(L, EL, BU);
  static constexpr int CH = LA * EL;
  static constexpr int RPC = CH / BU;  // columns advanced per step
  static_assert(CH % BU == 0, "chunk must hold whole columns");
};

// 16-byte load of matrix values with the nontemporal hint: the panels are
// read once per product, and keeping them out of the caches' working set
// leaves L2 to the x gathers of neighbouring rows
typedef double hf_double2v __attribute__((ext_vector_type(2)));
typedef float hf_float4v __attribute__((ext_vector_type(4)));
template <typename T>
__device__ inline typename Vec16<T>::type load_stream(const T *p);
template <>
__device__ inline double2 load_stream<double>(const double *p) {
  const hf_double2v v = __builtin_nontemporal_load((const hf_double2v *)p);
  return double2(v.x, v.y);
}
template <>
__device__ inline float4 load_stream<float>(const float *p) {
  const hf_float4v v = __builtin_nontemporal_load((const hf_float4v *)p);
  return float4(v.x, v.y, v.z, v.w);
}

template <typename T>
__device__ inline T vget(const typename Vec16<T>::type &v, int s);
template <>
__device__ inline double vget<double>(const double2 &v, int s) { return s == 0 ? v.x : v.y; }
template <>
__device__ inline float vget<float>(const float4 &v, int s) {
  return s == 0 ? v.x : (s == 1 ? v.y : (s == 2 ? v.z : v.w));
}

// Instance mask of the batched solver: a row of instance b is computed when
// mode = 0, when solving[b] (mode 1), or when solving[b] and kconv[b] < 0
// (mode 2, the instance still iterates in its cycle); other rows are left
// untouched.
struct RowMask {
  const int32_t *inst;  // instance of each element (or pressure node)
  const int *solving, *kconv;
  int mode;
  const uint8_t *skip = nullptr;  // rows left to another kernel (skip[r] != 0)
  __device__ bool live(int64_t r) const {
    if (skip && skip[r]) return false;
    if (!mode) return true;
    const int b = inst[r];
    return solving[b] != 0 && (mode == 1 || kconv[b] < 0);
  }
};

template <typename T, int BU, int LN, int NT, bool STRIPS>
__global__ __launch_bounds__(NT) void k_bsr_spmv(
    int64_t ne, const int64_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const T *__restrict__ A, const int64_t *__restrict__ sp_ptr,
    const int32_t *__restrict__ sp_pnode, const T *__restrict__ Bs, const T *__restrict__ x,
    const T *__restrict__ xp, T *__restrict__ y, RowMask mask, const T *__restrict__ add) {
  using S = SpmvShape<T, BU, LN>;
  constexpr int L = S::L, EL = S::EL, LA = S::LA, CH = S::CH, RPC = S::RPC, G = NT / L;
  using V = typename Vec16<T>::type;
  __shared__ T xs[G][5 * BU];
  __shared__ T part[G][CH];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int64_t e = (int64_t)blockIdx.x * G + g;
  const bool live = e < ne && mask.live(e);
  int64_t b0 = 0;
  int nb = 0;
  if (live) {
    b0 = blk_ptr[e];
    nb = (int)(blk_ptr[e + 1] - b0);
    // stage the x values of the row's (at most 5) block columns: the column
    // indices of all of a lane's entries first, then all their x loads
    constexpr int XT = (5 * BU + L - 1) / L;
    int32_t col[XT];
#pragma unroll
    for (int i = 0; i < XT; ++i) col[i] = blk_col[b0 + min((lane + L * i) / BU, nb - 1)];  // nb >= 1
    int64_t src[XT];
#pragma unroll
    for (int i = 0; i < XT; ++i) {
      const int t = lane + L * i;
      src[i] = t < nb * BU ? (int64_t)col[i] * BU + t % BU : -1;
    }
    T xv[XT];
#pragma unroll
    for (int i = 0; i < XT; ++i) xv[i] = src[i] >= 0 ? x[src[i]] : T(0);
#pragma unroll
    for (int i = 0; i < XT; ++i) {
      const int t = lane + L * i;
      if (t < nb * BU) xs[g][t] = xv[i];
    }
  }
  __syncthreads();
  T acc[EL];
#pragma unroll
  for (int s = 0; s < EL; ++s) acc[s] = T(0);
  if (live && lane < LA) {
    const T *panel = A + b0 * BU * BU;
    const int total = nb * BU * BU;
    int colS[EL];
#pragma unroll
    for (int s = 0; s < EL; ++s) colS[s] = (lane * EL + s) / BU;
    int f = lane * EL, cb = 0;
#pragma unroll 8
    for (; f < total; f += CH, cb += RPC) {
      const V v = load_stream<T>(panel + f);
#pragma unroll
      for (int s = 0; s < EL; ++s) acc[s] += vget<T>(v, s) * xs[g][cb + colS[s]];
    }
  }
  if (lane < LA) {
#pragma unroll
    for (int s = 0; s < EL; ++s) part[g][lane * EL + s] = acc[s];
  }
  __syncthreads();
  if (live && lane < BU) {
    T sum = T(0);
#pragma unroll
    for (int t = 0; t < RPC; ++t) sum += part[g][lane + BU * t];
    if (STRIPS) {
      for (int64_t k = sp_ptr[e]; k < sp_ptr[e + 1]; ++k) sum += Bs[k * BU + lane] * xp[sp_pnode[k]];
    }
    if (add) sum += add[e * BU + lane];
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
                                              T *__restrict__ yp, RowMask mask) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  if (!mask.live(i)) return;  // the whole wave leaves together
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

// element rows of the product with LN lanes per row
template <typename T, int BU, int LN, bool STRIPS>
static void rows_launch(int64_t ne, const int64_t *ptr, const int32_t *col, const T *A,
                        const int64_t *sp_ptr, const int32_t *sp_pnode, const T *Bs, const T *x,
                        const T *xp, T *y, const RowMask &me, hipStream_t st, const T *add = nullptr) {
  constexpr int NT = 256, G = NT / LN;
  hipLaunchKernelGGL((k_bsr_spmv<T, BU, LN, NT, STRIPS>), dim3((unsigned)((ne + G - 1) / G)), dim3(NT),
                     0, st, ne, ptr, col, A, sp_ptr, sp_pnode, Bs, x, xp, y, me, add);
}

template <typename T, int BU>
static void spmv_bu(const KParams &kp, const T *A, const T *Bs, const T *Cs, const T *D,
                    const T *x, T *y, const RowSel &sel, hipStream_t st) {
  const RowMask me{kp.einst, sel.solving, sel.kconv, sel.mode};
  const RowMask mp{kp.pinst, sel.solving, sel.kconv, sel.mode};
  constexpr int LW = wide_lanes(BU);
  const int64_t ne = kp.s.ne;
  if (ne) {
    if (kp.spmv_var == 1)
      rows_launch<T, BU, LW / 2, true>(ne, kp.m.blk_ptr, kp.m.blk_col, A, kp.m.sp_ptr, kp.m.sp_pnode,
                                       Bs, x, x + kp.s.n_u, y, me, st);
    else
      rows_launch<T, BU, LW, true>(ne, kp.m.blk_ptr, kp.m.blk_col, A, kp.m.sp_ptr, kp.m.sp_pnode, Bs,
                                   x, x + kp.s.n_u, y, me, st);
  }
  if (kp.s.n_p)
    hipLaunchKernelGGL((k_prows<T, BU>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.s.n_p,
                       kp.pinst, kp.poff, kp.doff, kp.m.pc_ptr, kp.m.pc_ent, kp.m.sp_elem, Cs, D, x,
                       x + kp.s.n_u, y + kp.s.n_u, mp);
}

template <typename T>
hipError_t launch_spmv(const KParams &kp, const T *A, const T *Bs, const T *Cs, const T *D,
                       const T *x, T *y, const RowSel &sel, hipStream_t st) {
  switch (kp.s.bu) {
    case 6: spmv_bu<T, 6>(kp, A, Bs, Cs, D, x, y, sel, st); break;
    case 12: spmv_bu<T, 12>(kp, A, Bs, Cs, D, x, y, sel, st); break;
    case 30: spmv_bu<T, 30>(kp, A, Bs, Cs, D, x, y, sel, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_spmv<double>(const KParams &, const double *, const double *,
                                        const double *, const double *, const double *,
                                        double *, const RowSel &, hipStream_t);
template hipError_t launch_spmv<float>(const KParams &, const float *, const float *,
                                       const float *, const float *, const float *, float *,
                                       const RowSel &, hipStream_t);

// element rows without strips or pressure rows, rows with skip[e] != 0 left
// to another kernel (the residual rows of the crack-free elements in an
// incremental assembly)
hipError_t launch_spmv_rows(const KParams &kp, const double *A, const double *x, double *y,
                            const uint8_t *skip, hipStream_t st) {
  RowMask me{kp.einst, nullptr, nullptr, 0};
  me.skip = skip;
  if (!kp.s.ne) return hipSuccess;
  switch (kp.s.bu) {
    case 6:
      rows_launch<double, 6, wide_lanes(6), false>(kp.s.ne, kp.m.blk_ptr, kp.m.blk_col, A, nullptr, nullptr,
                                                   nullptr, x, nullptr, y, me, st);
      break;
    case 12:
      rows_launch<double, 12, wide_lanes(12), false>(kp.s.ne, kp.m.blk_ptr, kp.m.blk_col, A, nullptr, nullptr,
                                                     nullptr, x, nullptr, y, me, st);
      break;
    case 30:
      rows_launch<double, 30, wide_lanes(30), false>(kp.s.ne, kp.m.blk_ptr, kp.m.blk_col, A, nullptr, nullptr,
                                                     nullptr, x, nullptr, y, me, st);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Residual r = b - J x with compensated (double-double) accumulation: every
// product a x is split exactly into p + e (two-product by FMA), the row sums
// carry their rounding errors (two-sum), and the difference with b is
// rounded once.  The computed residual is then accurate to about u ||r|| +
// u^2 ||J|| ||x|| instead of u ||J|| ||x||, so a relative residual below
// u ||J|| ||x|| / ||b|| stays attainable when the solution is large against
// the right-hand side (late Newton iterations of ill-conditioned systems).
// ---------------------------------------------------------------------------
struct DD {
  double hi, lo;
};
__device__ inline void dd_add(DD &s, double v) {  // s += v (two-sum, error kept in lo)
#pragma clang fp contract(off)
  const double t = s.hi + v;
  const double bp = t - s.hi;
  s.lo += (s.hi - (t - bp)) + (v - bp);
  s.hi = t;
}
__device__ inline void dd_fma(DD &s, double a, double b) {  // s += a b
#pragma clang fp contract(off)
  const double p = a * b;
  const double e = fma(a, b, -p);
  dd_add(s, p);
  s.lo += e;
}
__device__ inline void dd_merge(DD &s, const DD &o) {  // s += o
  dd_add(s, o.hi);
  s.lo += o.lo;
}
__device__ inline double dd_sub_from(double b, const DD &s) {  // b - s, rounded once
#pragma clang fp contract(off)
  DD t{b, 0.0};
  dd_add(t, -s.hi);
  return t.hi + (t.lo - s.lo);
}

template <int BU, int LN, int NT>
__global__ __launch_bounds__(NT) void k_bsr_resid(
    int64_t ne, const int64_t *__restrict__ blk_ptr, const int32_t *__restrict__ blk_col,
    const double *__restrict__ A, const int64_t *__restrict__ sp_ptr,
    const int32_t *__restrict__ sp_pnode, const double *__restrict__ Bs, const double *__restrict__ x,
    const double *__restrict__ xp, const double *__restrict__ bvec, double *__restrict__ r, RowMask mask) {
  using S = SpmvShape<double, BU, LN>;
  constexpr int L = S::L, EL = S::EL, LA = S::LA, CH = S::CH, RPC = S::RPC, G = NT / L;
  __shared__ double xs[G][5 * BU];
  __shared__ double ph[G][CH], pl[G][CH];
  const int g = threadIdx.x / L, lane = threadIdx.x % L;
  const int64_t e = (int64_t)blockIdx.x * G + g;
  const bool live = e < ne && mask.live(e);
  int64_t b0 = 0;
  int nb = 0;
  if (live) {
    b0 = blk_ptr[e];
    nb = (int)(blk_ptr[e + 1] - b0);
    for (int t = lane; t < nb * BU; t += L) xs[g][t] = x[(int64_t)blk_col[b0 + t / BU] * BU + t % BU];
  }
  __syncthreads();
  DD acc[EL];
#pragma unroll
  for (int s2 = 0; s2 < EL; ++s2) acc[s2] = DD{0.0, 0.0};
  if (live && lane < LA) {
    const double *panel = A + b0 * BU * BU;
    const int total = nb * BU * BU;
    int colS[EL];
#pragma unroll
    for (int s2 = 0; s2 < EL; ++s2) colS[s2] = (lane * EL + s2) / BU;
    int f = lane * EL, cb = 0;
#pragma unroll 4
    for (; f < total; f += CH, cb += RPC) {
      const double2 v = load_stream<double>(panel + f);
      dd_fma(acc[0], v.x, xs[g][cb + colS[0]]);
      dd_fma(acc[1], v.y, xs[g][cb + colS[1]]);
    }
  }
  if (lane < LA) {
#pragma unroll
    for (int s2 = 0; s2 < EL; ++s2) {
      ph[g][lane * EL + s2] = acc[s2].hi;
      pl[g][lane * EL + s2] = acc[s2].lo;
    }
  }
  __syncthreads();
  if (live && lane < BU) {
    DD sum{0.0, 0.0};
#pragma unroll
    for (int t = 0; t < RPC; ++t) dd_merge(sum, DD{ph[g][lane + BU * t], pl[g][lane + BU * t]});
    for (int64_t k = sp_ptr[e]; k < sp_ptr[e + 1]; ++k) dd_fma(sum, Bs[k * BU + lane], xp[sp_pnode[k]]);
    const int64_t row = e * BU + lane;
    r[row] = dd_sub_from(bvec[row], sum);
  }
}

// pressure rows of the compensated residual (one wave per row)
template <int BU>
__global__ __launch_bounds__(64) void k_presid(int64_t np, const int32_t *__restrict__ pinst,
                                               const int32_t *__restrict__ poff,
                                               const int64_t *__restrict__ doff,
                                               const int32_t *__restrict__ pc_ptr,
                                               const int32_t *__restrict__ pc_ent,
                                               const int32_t *__restrict__ sp_elem,
                                               const double *__restrict__ Cs, const double *__restrict__ D,
                                               const double *__restrict__ xu, const double *__restrict__ xp,
                                               const double *__restrict__ bp, double *__restrict__ rp,
                                               RowMask mask) {
  __shared__ double sh[64], sl[64];
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  if (!mask.live(i)) return;  // the whole wave leaves together
  DD acc{0.0, 0.0};
  if (pc_ptr) {
    for (int32_t c = pc_ptr[i]; c < pc_ptr[i + 1]; ++c) {
      const int32_t ent = pc_ent[c];
      const int64_t e = sp_elem[ent];
      if (lane < BU) dd_fma(acc, Cs[(int64_t)ent * BU + lane], xu[e * BU + lane]);
    }
  }
  const int b = pinst[i];
  const int64_t p0 = poff[b], nb = poff[b + 1] - p0;
  const double *Drow = D + doff[b] + (i - p0) * nb;
  for (int64_t j = lane; j < nb; j += 64) dd_fma(acc, Drow[j], xp[p0 + j]);
  sh[lane] = acc.hi;
  sl[lane] = acc.lo;
  __syncthreads();
  if (lane == 0) {
    DD tot{0.0, 0.0};
    for (int t = 0; t < 64; ++t) dd_merge(tot, DD{sh[t], sl[t]});
    rp[i] = dd_sub_from(bp[i], tot);
  }
}

template <int BU>
static void resid_bu(const KParams &kp, const double *A, const double *Bs, const double *Cs, const double *D,
                     const double *x, const double *b, double *r, const RowSel &sel, hipStream_t st) {
  const RowMask me{kp.einst, sel.solving, sel.kconv, sel.mode};
  const RowMask mp{kp.pinst, sel.solving, sel.kconv, sel.mode};
  constexpr int LW = wide_lanes(BU), NT = 256, G = NT / LW;
  const int64_t ne = kp.s.ne;
  if (ne)
    hipLaunchKernelGGL((k_bsr_resid<BU, LW, NT>), dim3((unsigned)((ne + G - 1) / G)), dim3(NT), 0, st, ne,
                       kp.m.blk_ptr, kp.m.blk_col, A, kp.m.sp_ptr, kp.m.sp_pnode, Bs, x, x + kp.s.n_u, b, r,
                       me);
  if (kp.s.n_p)
    hipLaunchKernelGGL((k_presid<BU>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.s.n_p, kp.pinst,
                       kp.poff, kp.doff, kp.m.pc_ptr, kp.m.pc_ent, kp.m.sp_elem, Cs, D, x, x + kp.s.n_u,
                       b + kp.s.n_u, r + kp.s.n_u, mp);
}

hipError_t launch_resid(const KParams &kp, const double *A, const double *Bs, const double *Cs, const double *D,
                        const double *x, const double *b, double *r, const RowSel &sel, hipStream_t st) {
  switch (kp.s.bu) {
    case 6: resid_bu<6>(kp, A, Bs, Cs, D, x, b, r, sel, st); break;
    case 12: resid_bu<12>(kp, A, Bs, Cs, D, x, b, r, sel, st); break;
    case 30: resid_bu<30>(kp, A, Bs, Cs, D, x, b, r, sel, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// folded product y = J M^-1 x: the pressure part of M^-1 first (t_p = S^-1
// x_p), then the row panels of A M_A^-1 with the B strips on t_p, then the
// pressure rows with the folded C strips and D on t_p
template <typename T, int BU>
static void spmv_folded_bu(const KParams &kp, const T *Af, const T *Bs, const T *Cf, const T *D,
                           const T *Sinv, const T *x, T *y, T *tp, const RowSel &sel, hipStream_t st) {
  const RowMask me{kp.einst, sel.solving, sel.kconv, sel.mode};
  const RowMask mp{kp.pinst, sel.solving, sel.kconv, sel.mode};
  constexpr int LW = wide_lanes(BU);
  const int64_t ne = kp.s.ne;
  if (kp.s.n_p)
    hipLaunchKernelGGL((k_prows<T, BU>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.s.n_p, kp.pinst,
                       kp.poff, kp.doff, nullptr, nullptr, nullptr, nullptr, Sinv, x + kp.s.n_u,
                       x + kp.s.n_u, tp, mp);
  if (ne) {
    if (kp.spmv_var == 1)
      rows_launch<T, BU, LW / 2, true>(ne, kp.m.blk_ptr, kp.m.blk_col, Af, kp.m.sp_ptr, kp.m.sp_pnode,
                                       Bs, x, tp, y, me, st);
    else
      rows_launch<T, BU, LW, true>(ne, kp.m.blk_ptr, kp.m.blk_col, Af, kp.m.sp_ptr, kp.m.sp_pnode, Bs,
                                   x, tp, y, me, st);
  }
  if (kp.s.n_p)
    hipLaunchKernelGGL((k_prows<T, BU>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.s.n_p,
                       kp.pinst, kp.poff, kp.doff, kp.m.pc_ptr, kp.m.pc_ent, kp.m.sp_elem, Cf, D, x,
                       tp, y + kp.s.n_u, mp);
}

template <typename T, int BU>
static void folded_rows_bu(const KParams &kp, const T *Af, const T *Bs, const T *x, const T *tp, const T *add, T *y,
                           hipStream_t st) {
  const RowMask me{kp.einst, nullptr, nullptr, 0};
  constexpr int LW = wide_lanes(BU);
  if (!kp.s.ne) return;
  if (kp.spmv_var == 1)
    rows_launch<T, BU, LW / 2, true>(kp.s.ne, kp.m.blk_ptr, kp.m.blk_col, Af, kp.m.sp_ptr, kp.m.sp_pnode, Bs, x,
                                     tp, y, me, st, add);
  else
    rows_launch<T, BU, LW, true>(kp.s.ne, kp.m.blk_ptr, kp.m.blk_col, Af, kp.m.sp_ptr, kp.m.sp_pnode, Bs, x, tp,
                                 y, me, st, add);
}

template <typename T>
hipError_t launch_spmv_folded_rows(const KParams &kp, const T *Af, const T *Bs, const T *x, const T *tp,
                                   const T *add, T *y, hipStream_t st) {
  switch (kp.s.bu) {
    case 6: folded_rows_bu<T, 6>(kp, Af, Bs, x, tp, add, y, st); break;
    case 12: folded_rows_bu<T, 12>(kp, Af, Bs, x, tp, add, y, st); break;
    case 30: folded_rows_bu<T, 30>(kp, Af, Bs, x, tp, add, y, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_spmv_folded_rows<double>(const KParams &, const double *, const double *,
                                                    const double *, const double *, const double *, double *,
                                                    hipStream_t);
template hipError_t launch_spmv_folded_rows<float>(const KParams &, const float *, const float *, const float *,
                                                   const float *, const float *, float *, hipStream_t);

template <typename T>
hipError_t launch_spmv_folded(const KParams &kp, const T *Af, const T *Bs, const T *Cf, const T *D,
                              const T *Sinv, const T *x, T *y, T *tp, const RowSel &sel, hipStream_t st) {
  switch (kp.s.bu) {
    case 6: spmv_folded_bu<T, 6>(kp, Af, Bs, Cf, D, Sinv, x, y, tp, sel, st); break;
    case 12: spmv_folded_bu<T, 12>(kp, Af, Bs, Cf, D, Sinv, x, y, tp, sel, st); break;
    case 30: spmv_folded_bu<T, 30>(kp, Af, Bs, Cf, D, Sinv, x, y, tp, sel, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_spmv_folded<double>(const KParams &, const double *, const double *,
                                               const double *, const double *, const double *,
                                               const double *, double *, double *, const RowSel &,
                                               hipStream_t);
template hipError_t launch_spmv_folded<float>(const KParams &, const float *, const float *, const float *,
                                              const float *, const float *, const float *, float *,
                                              float *, const RowSel &, hipStream_t);

// block-Jacobi apply: z_u = blockdiag(inv) r_u (the same streaming kernel on
// the identity block pattern), z_p = S^-1 r_p
template <typename T, int BU>
static void precond_bu(const KParams &kp, const T *inv, const T *Sinv, const T *r, T *z,
                       const RowSel &sel, hipStream_t st, const int64_t *ident_ptr,
                       const int32_t *ident_col) {
  const RowMask me{kp.einst, sel.solving, sel.kconv, sel.mode};
  const RowMask mp{kp.pinst, sel.solving, sel.kconv, sel.mode};
  constexpr int LW = wide_lanes(BU);
  const int64_t ne = kp.s.ne;
  if (ne) {
    if (kp.prec_var == 1)
      rows_launch<T, BU, LW / 2, false>(ne, ident_ptr, ident_col, inv, nullptr, nullptr, nullptr, r,
                                        nullptr, z, me, st);
    else
      rows_launch<T, BU, LW, false>(ne, ident_ptr, ident_col, inv, nullptr, nullptr, nullptr, r,
                                    nullptr, z, me, st);
  }
  if (kp.s.n_p)
    hipLaunchKernelGGL((k_prows<T, BU>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp.s.n_p,
                       kp.pinst, kp.poff, kp.doff, nullptr, nullptr, nullptr, nullptr, Sinv, r,
                       r + kp.s.n_u, z + kp.s.n_u, mp);
}

template <typename T>
hipError_t launch_precond(const KParams &kp, const T *inv, const T *Sinv, const T *r, T *z,
                          const RowSel &sel, hipStream_t st) {
  const int64_t *ip = kp.m.ident_ptr;
  const int32_t *ic = kp.m.ident_col;
  switch (kp.s.bu) {
    case 6: precond_bu<T, 6>(kp, inv, Sinv, r, z, sel, st, ip, ic); break;
    case 12: precond_bu<T, 12>(kp, inv, Sinv, r, z, sel, st, ip, ic); break;
    case 30: precond_bu<T, 30>(kp, inv, Sinv, r, z, sel, st, ip, ic); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
template hipError_t launch_precond<double>(const KParams &, const double *, const double *,
                                           const double *, double *, const RowSel &, hipStream_t);
template hipError_t launch_precond<float>(const KParams &, const float *, const float *,
                                          const float *, float *, const RowSel &, hipStream_t);

// ---------------------------------------------------------------------------
// Scratch of the allocation-free folded product: the S^-1 x_p staging vector
// of launch_spmv_folded in a file-scope device array instead of a context
// buffer.  Each GPU holds its own copy of the array; its address on a device
// is looked up once (with that device current) and kept.  Every caller on a
// GPU shares the array: calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[kNoAllocScratchElems];

hipError_t noalloc_scratch(int device, void **ptr) {
  static std::mutex mu;
  static std::vector<void *> per_device;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((int)per_device.size() <= device) per_device.resize(device + 1, nullptr);
  if (!per_device[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[device] = p;
  }
  *ptr = per_device[device];
  return hipSuccess;
}

}  // namespace hf
