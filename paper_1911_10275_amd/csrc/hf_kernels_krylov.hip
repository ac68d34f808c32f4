// Batched Krylov kernels for gfx950: GMRES vector work segmented by
// instance, and the per-instance Hessenberg / Givens / least-squares steps
// on the device, so that a chunk of GMRES iterations runs without host
// round trips (and can be captured in a HIP graph).
//
// Row chunks.  The rows of the global vector [u_all; p_all] are cut into
// chunks of at most KC_CHUNK rows that never straddle two instances; chunk c
// covers rows [row0[c], row0[c] + len[c]) of instance inst[c], and the
// chunks of instance b are [cptr[b], cptr[b+1]).  Each chunk writes one
// partial per output; k_seg_reduce sums the partials of an instance in a
// fixed order, so every reduction is bitwise reproducible.
//
// Instance state (one entry per instance): solving[b] (1 while the instance
// still iterates in this cycle), kconv[b] (-1, or the basis size at which the
// cycle stopped), bnorm[b], H[b] ((m+1) x m, row-major), cs/sn[b] (m), g[b]
// (m+1), scale[b] (1/||w|| used to normalise the next basis vector).
#include <cmath>

#include "hf_internal.h"

namespace hf {

constexpr int KT = 256;        // threads per block of the vector kernels
constexpr int KTILE = 8;       // basis vectors per tile of the Gram-Schmidt passes

// Wavefront sum without LDS round trips: two quad permutes and two row
// rotations (DPP) give every lane the sum of its row of 16 lanes, and the
// four row sums are read from lanes 0, 16, 32 and 48 in a fixed order.  The
// whole wavefront must be active; every lane receives the total.
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double lane_f64(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline double kwave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x128>(v);  // row_ror:8
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

__device__ inline bool inst_on(const KrylovDev &kd, int b) {
  return kd.solving[b] != 0 && kd.kconv[b] < 0;
}

// partial[c*(k+1) + i] = chunk sum of V_i w (i < k); partial[c*(k+1) + k] = chunk sum of w^2.
// With gate != nullptr the chunk only works when gate[inst] != 0.
// Each wavefront covers all rows of the chunk (KRL rows per lane, w held in
// registers) for the basis vectors i = wave, wave + NW, ...: per vector a
// lane issues its KRL loads at once and one wavefront sum gives the dot, so
// there is no cross-wave combination; two vectors are in flight at a time.
constexpr int KRL = kChunkRows / 64;  // rows per lane of a wavefront-wide chunk

// Load of a basis entry by the Gram-Schmidt passes: FP64 bases (m+1 vectors
// of N doubles, far beyond the caches at full size) are streamed with the
// nontemporal hint; FP32 bases use plain loads, which measured faster there.
template <typename T>
__device__ inline T ld_basis(const T *p) {
  if constexpr (sizeof(T) == 8)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <typename T, int RR>
__global__ __launch_bounds__(kChunkRows / RR) void k_sproj(KrylovDev kd, const T *__restrict__ V, int64_t ldv,
                                                           int k, const T *__restrict__ w,
                                                           const int *__restrict__ gate,
                                                           double *__restrict__ partial) {
  constexpr int NTH = kChunkRows / RR, NW = NTH / 64;
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int b = kd.c_inst[c];
  double *out = partial + (int64_t)c * (k + 1);
  if (!inst_on(kd, b) || (gate && !gate[b])) {
    for (int i = tid; i <= k; i += NTH) out[i] = 0.0;
    return;
  }
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  double wr[KRL];
#pragma unroll
  for (int s = 0; s < KRL; ++s) {
    const int rr = lane + 64 * s;
    wr[s] = rr < len ? (double)w[row0 + rr] : 0.0;
  }
  if (wv == NW - 1) {
    double nn = 0.0;
#pragma unroll
    for (int s = 0; s < KRL; ++s) nn += wr[s] * wr[s];
    nn = kwave_sum(nn);
    if (lane == 0) out[k] = nn;
  }
  // VF basis vectors per wavefront pass (their loads are issued together)
  constexpr int VF = 2;
  int i = wv;
  for (; i + (VF - 1) * NW < k; i += VF * NW) {
    // all loads of the pass first (rows past len read the last row: wr is 0
    // there), then the products
    T x[VF][KRL];
#pragma unroll
    for (int s = 0; s < KRL; ++s) {
      const int rc = min(lane + 64 * s, len - 1);
#pragma unroll
      for (int f = 0; f < VF; ++f) x[f][s] = ld_basis(&V[(int64_t)(i + f * NW) * ldv + row0 + rc]);
    }
    double a[VF];
#pragma unroll
    for (int f = 0; f < VF; ++f) a[f] = 0.0;
#pragma unroll
    for (int s = 0; s < KRL; ++s)
#pragma unroll
      for (int f = 0; f < VF; ++f) a[f] += (double)x[f][s] * wr[s];
#pragma unroll
    for (int f = 0; f < VF; ++f) {
      const double t = kwave_sum(a[f]);
      if (lane == 0) out[i + f * NW] = t;
    }
  }
  for (; i < k; i += NW) {
    const T *va = V + (int64_t)i * ldv + row0;
    double a0 = 0.0;
#pragma unroll
    for (int s = 0; s < KRL; ++s) a0 += (double)ld_basis(&va[min(lane + 64 * s, len - 1)]) * wr[s];
    a0 = kwave_sum(a0);
    if (lane == 0) out[i] = a0;
  }
}

// w -= V h_b (h_b = h + b*hstride); partial[c] = chunk sum of the new w^2.
template <typename T, int RR>
__global__ __launch_bounds__(kChunkRows / RR) void k_supdate(KrylovDev kd, const T *__restrict__ V, int64_t ldv,
                                                int k, const double *__restrict__ h, int hstride,
                                                T *__restrict__ w, const int *__restrict__ gate,
                                                double *__restrict__ partial) {
  constexpr int NTH = kChunkRows / RR;
  __shared__ double sh[kMaxKrylov];
  __shared__ double wsum[NTH / 64];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int b = kd.c_inst[c];
  if (!inst_on(kd, b) || (gate && !gate[b])) {
    if (tid == 0) partial[c] = 0.0;
    return;
  }
  for (int i = tid; i < k; i += NTH) sh[i] = h[(int64_t)b * hstride + i];
  __syncthreads();
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  double acc[RR];
#pragma unroll
  for (int s = 0; s < RR; ++s) {
    const int rr = tid + s * NTH;
    acc[s] = rr < len ? (double)w[row0 + rr] : 0.0;
  }
  // basis vectors per tile: twice as many in FP32 (the same bytes per
  // lane).  The loads of a tile are issued together; rows past len read the
  // chunk's last row and are never stored.
  constexpr int TW = sizeof(T) == 4 ? 2 * KTILE : KTILE;
  int rc[RR];
#pragma unroll
  for (int s = 0; s < RR; ++s) rc[s] = min(tid + s * NTH, len - 1);
  int i0 = 0;
  for (; i0 + TW <= k; i0 += TW) {
    T x[TW][RR];
#pragma unroll
    for (int q = 0; q < TW; ++q)
#pragma unroll
      for (int s = 0; s < RR; ++s) x[q][s] = ld_basis(&V[(int64_t)(i0 + q) * ldv + row0 + rc[s]]);
#pragma unroll
    for (int s = 0; s < RR; ++s)
#pragma unroll
      for (int q = 0; q < TW; ++q) acc[s] -= sh[i0 + q] * (double)x[q][s];
  }
  for (; i0 < k; ++i0) {
#pragma unroll
    for (int s = 0; s < RR; ++s) acc[s] -= sh[i0] * (double)ld_basis(&V[(int64_t)i0 * ldv + row0 + rc[s]]);
  }
  double nn = 0.0;
#pragma unroll
  for (int s = 0; s < RR; ++s) {
    const int rr = tid + s * NTH;
    if (rr < len) {
      const T v = (T)acc[s];
      w[row0 + rr] = v;
      nn += (double)v * (double)v;
    }
  }
  nn = kwave_sum(nn);
  if (lane == 0) wsum[wv] = nn;
  __syncthreads();
  if (tid == 0) {
    double s2 = 0.0;
    for (int q = 0; q < NTH / 64; ++q) s2 += wsum[q];
    partial[c] = s2;
  }
}

// One-reduce projection of the single-pass (inverse compact WY) modified
// Gram-Schmidt: with k = j+1 basis vectors and v_j = V_{k-1},
// partial[c*nout + i] = chunk sum of V_i w (i < k) and
// partial[c*nout + k + l] = chunk sum of V_l v_j (l < k-1); nout = 2k - 1.
// Wavefront-per-vector as in k_sproj; w and v_j are staged in LDS (FP64) so
// that the registers hold the loads of two basis vectors in flight.
template <typename T, int RR>
__global__ __launch_bounds__(kChunkRows / RR) void k_sproj2(KrylovDev kd, const T *__restrict__ V,
                                                            int64_t ldv, int k,
                                                            const T *__restrict__ w,
                                                            double *__restrict__ partial) {
  constexpr int NTH = kChunkRows / RR, NW = NTH / 64;
  __shared__ double s_w[kChunkRows], s_v[kChunkRows];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int b = kd.c_inst[c];
  const int nout = 2 * k - 1;
  double *out = partial + (int64_t)c * nout;
  if (!inst_on(kd, b)) {
    for (int i = tid; i < nout; i += NTH) out[i] = 0.0;
    return;
  }
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  const T *vj = V + (int64_t)(k - 1) * ldv + row0;
  for (int r = tid; r < kChunkRows; r += NTH) {
    s_w[r] = r < len ? (double)w[row0 + r] : 0.0;
    s_v[r] = r < len ? (double)vj[r] : 0.0;
  }
  __syncthreads();
  int i = wv;
  for (; i + NW < k; i += 2 * NW) {
    const T *va = V + (int64_t)i * ldv + row0, *vb = va + (int64_t)NW * ldv;
    // keep the compiler from holding w and v_j in registers across passes
    // (that leaves too few for the loads in flight): they are re-read from
    // LDS after the loads of the pass are issued
    __asm__ volatile("" ::: "memory");
    T xa[KRL], xb[KRL];
#pragma unroll
    for (int s = 0; s < KRL; ++s) {
      const int rc = min(lane + 64 * s, len - 1);  // s_w, s_v are 0 past len
      xa[s] = ld_basis(&va[rc]);
      xb[s] = ld_basis(&vb[rc]);
    }
    double aw = 0.0, av = 0.0, bw = 0.0, bv = 0.0;
#pragma unroll
    for (int s = 0; s < KRL; ++s) {
      const int rr = lane + 64 * s;
      const double x = (double)xa[s], y = (double)xb[s];
      const double ws = s_w[rr], vs = s_v[rr];
      aw += x * ws;
      av += x * vs;
      bw += y * ws;
      bv += y * vs;
    }
    aw = kwave_sum(aw);
    av = kwave_sum(av);
    bw = kwave_sum(bw);
    bv = kwave_sum(bv);
    if (lane == 0) {
      out[i] = aw;
      out[k + i] = av;  // i + NW < k, so i < k - 1
      out[i + NW] = bw;
      if (i + NW < k - 1) out[k + i + NW] = bv;
    }
  }
  for (; i < k; i += NW) {
    const T *va = V + (int64_t)i * ldv + row0;
    double aw = 0.0, av = 0.0;
#pragma unroll
    for (int s = 0; s < KRL; ++s) {
      const int rr = lane + 64 * s;
      const double x = (double)ld_basis(&va[min(rr, len - 1)]);
      aw += x * s_w[rr];
      av += x * s_v[rr];
    }
    aw = kwave_sum(aw);
    av = kwave_sum(av);
    if (lane == 0) {
      out[i] = aw;
      if (i < k - 1) out[k + i] = av;
    }
  }
}

// Coefficients of the single-pass modified Gram-Schmidt from one reduction:
// row j of the strictly lower Gram factor, L[j][l] = v_j . v_l (l < j), is
// stored; h solves (I + L) h = s (s_i = v_i . w, i <= j) by forward
// substitution, which reproduces the projections of the sequential
// (modified) Gram-Schmidt.  L is stored packed by rows (row i, of length i,
// at i (i - 1) / 2), so rows 1 .. j-1 are one contiguous range.  One
// wavefront per iterating instance; for j < 64 the factor is staged in LDS
// (eight loads in flight per lane) and eliminated column by column.
constexpr int kIcwyLds = 64;
__device__ inline int lrow(int i) { return i * (i - 1) / 2; }
__global__ __launch_bounds__(64) void k_icwy(KrylovDev kd, int j, int m, const double *__restrict__ sv,
                                             double *__restrict__ Lmat, double *__restrict__ h,
                                             int hstride) {
  __shared__ double hs[kMaxKrylov];
  __shared__ double Lp[kIcwyLds * (kIcwyLds - 1) / 2];
  const int b = blockIdx.x, lane = threadIdx.x;
  if (!inst_on(kd, b)) return;  // uniform over the block
  const int k = j + 1, nout = 2 * k - 1, ld = m + 1;
  const double *sb = sv + (int64_t)b * nout;
  double *Lb = Lmat + (int64_t)b * ld * ld;
  for (int l = lane; l < j; l += 64) Lb[lrow(j) + l] = sb[k + l];
  for (int i = lane; i <= j; i += 64) hs[i] = sb[i];
  if (j < kIcwyLds) {
    constexpr int U = 8;
    const int n = lrow(j);
    for (int t0 = 0; t0 < n; t0 += 64 * U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + 64 * u + lane;
        v[u] = t < n ? Lb[t] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = t0 + 64 * u + lane;
        if (t < n) Lp[t] = v[u];
      }
    }
    for (int l = lane; l < j; l += 64) Lp[n + l] = sb[k + l];
    __syncthreads();
    for (int l = 0; l < j; ++l) {  // h_l is final: remove it from the rows below
      const double hl = hs[l];
      const int i = l + 1 + lane;
      if (i <= j) hs[i] -= Lp[lrow(i) + l] * hl;
      __syncthreads();
    }
  } else {
    __syncthreads();
    for (int i = 0; i <= j; ++i) {
      const double *Li = i == j ? sb + k : Lb + lrow(i);  // row i of L (row j from sv)
      double acc = 0.0;
      for (int l = lane; l < i; l += 64) acc += Li[l] * hs[l];
      acc = kwave_sum(acc);
      if (lane == 0) hs[i] -= acc;
      __syncthreads();
    }
  }
  double *hb = h + (int64_t)b * hstride;
  for (int i = lane; i <= j; i += 64) hb[i] = hs[i];
}

// out[b*nout + i] = sum over the chunks of instance b of partial[c*nout + i]
__global__ __launch_bounds__(KT) void k_seg_reduce(KrylovDev kd, const double *__restrict__ partial,
                                                   int nout, double *__restrict__ out) {
  __shared__ double sm[KT];
  const int b = blockIdx.x, i = blockIdx.y;
  const int c0 = kd.cptr[b], c1 = kd.cptr[b + 1];
  double acc = 0.0;
  for (int c = c0 + threadIdx.x; c < c1; c += KT) acc += partial[(int64_t)c * nout + i];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = KT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)b * nout + i] = sm[0];
}

// v[r] = w[r] * scale[inst] for instances with a non-zero scale (the others,
// not iterating, keep whatever their rows hold: no kernel reads them)
template <typename T>
__global__ __launch_bounds__(KT) void k_sscale(KrylovDev kd, const T *__restrict__ w,
                                               const double *__restrict__ scale, T *__restrict__ v) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = kd.c_inst[c];
  const double s = kd.solving[b] ? scale[b] : 0.0;
  if (s == 0.0) return;  // idle instance: its basis rows are never read
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  for (int rr = tid; rr < len; rr += KT) v[row0 + rr] = (T)((double)w[row0 + rr] * s);
}

// out[r] = sum_{i < nb} y_b[i] V_i[r], nb = basis size of the instance's cycle
template <typename T>
__global__ __launch_bounds__(KT) void k_scombine(KrylovDev kd, const T *__restrict__ V, int64_t ldv,
                                                 const double *__restrict__ y, int ystride,
                                                 const int *__restrict__ nbasis, T *__restrict__ out) {
  __shared__ double sy[kMaxKrylov];
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = kd.c_inst[c];
  const int nb = kd.solving[b] ? nbasis[b] : 0;
  for (int i = tid; i < nb; i += KT) sy[i] = y[(int64_t)b * ystride + i];
  __syncthreads();
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  for (int rr = tid; rr < len; rr += KT) {
    double acc = 0.0;
    for (int i = 0; i < nb; ++i) acc += sy[i] * (double)V[(int64_t)i * ldv + row0 + rr];
    out[row0 + rr] = (T)acc;
  }
}

// x[r] += a_b * z[r]  (a_b = coef[inst] or 1 when coef is null; only iterating instances)
template <typename TX, typename TZ>
__global__ __launch_bounds__(KT) void k_saxpy(KrylovDev kd, const double *__restrict__ coef,
                                              const TZ *__restrict__ z, TX *__restrict__ x) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = kd.c_inst[c];
  if (!kd.solving[b]) return;
  const double a = coef ? coef[b] : 1.0;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  for (int rr = tid; rr < len; rr += KT) x[row0 + rr] = (TX)((double)x[row0 + rr] + a * (double)z[row0 + rr]);
}

// r = b - Jx for iterating instances (others untouched)
template <typename T>
__global__ __launch_bounds__(KT) void k_ssub(KrylovDev kd, const T *__restrict__ bvec,
                                             const T *__restrict__ jx, T *__restrict__ r) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = kd.c_inst[c];
  if (!kd.solving[b]) return;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  for (int rr = tid; rr < len; rr += KT) r[row0 + rr] = bvec[row0 + rr] - jx[row0 + rr];
}

// y[r] = (T)(x[r] * coef[inst])  (precision cast with per-instance scale; 0 when idle)
template <typename TY, typename TX>
__global__ __launch_bounds__(KT) void k_scast(KrylovDev kd, const TX *__restrict__ x,
                                              const double *__restrict__ coef, TY *__restrict__ y) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = kd.c_inst[c];
  const double a = kd.solving[b] ? coef[b] : 0.0;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  for (int rr = tid; rr < len; rr += KT) y[row0 + rr] = a == 0.0 ? TY(0) : (TY)(a * (double)x[row0 + rr]);
}

// y[r] = x[r] on the rows of iterating instances (other instances untouched)
template <typename T>
__global__ __launch_bounds__(KT) void k_scopy(KrylovDev kd, const T *__restrict__ x, T *__restrict__ y) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = kd.c_inst[c];
  if (!kd.solving[b]) return;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  for (int rr = tid; rr < len; rr += KT) y[row0 + rr] = x[row0 + rr];
}

// zero a vector segment-wise (graph-safe replacement of memset)
template <typename T>
__global__ __launch_bounds__(KT) void k_szero(KrylovDev kd, T *__restrict__ x, int only_solving) {
  const int c = blockIdx.x, tid = threadIdx.x;
  const int b = kd.c_inst[c];
  if (only_solving && !kd.solving[b]) return;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  for (int rr = tid; rr < len; rr += KT) x[row0 + rr] = T(0);
}

// Re-orthogonalisation test (Daniel-Gragg-Kaufman-Stewart): flag[b] = 1 when
// ||w1|| < ||w|| / sqrt(2).  n0 = ||w||^2 (stride n0s), n1 = ||w1||^2.
// policy 0: the test; 1: always (every iterating instance); 2: never
__global__ void k_reorth_flag(KrylovDev kd, const double *__restrict__ n0, int n0s,
                              const double *__restrict__ n1, int policy, int *__restrict__ flag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= kd.n_inst) return;
  const bool test = policy == 1 || (policy == 0 && n1[b] < 0.5 * n0[(int64_t)b * n0s]);
  flag[b] = inst_on(kd, b) && test ? 1 : 0;
}

// Arnoldi step j of every iterating instance: column j of H from the two
// Gram-Schmidt passes, previous rotations, the new rotation, the residual
// estimate; stop the cycle of an instance when the estimate reaches
// rtol[b] * bnorm[b], on breakdown, or at its iteration cap.
// One wavefront per instance: the lanes gather column j of H (both passes)
// and the previous rotations into LDS, lane 0 applies the rotations in
// sequence (the column entry being rotated stays in a register), and the
// lanes write the column back.
__global__ __launch_bounds__(64) void k_arnoldi(KrylovDev kd, int j, int m,
                                                const double *__restrict__ s1, int s1s,
                                                const double *__restrict__ s2, int s2s,
                                                const int *__restrict__ reorth,
                                                const double *__restrict__ n1,
                                                const double *__restrict__ n2,
                                                const double *__restrict__ pnorm,
                                                double *__restrict__ scale) {
  __shared__ double col[kMaxKrylov + 1], c_s[kMaxKrylov], s_s[kMaxKrylov];
  __shared__ double s_nn;
  const int b = blockIdx.x, lane = threadIdx.x;
  if (!inst_on(kd, b)) {  // uniform over the block
    if (lane == 0) scale[b] = 0.0;
    return;
  }
  // ||w||^2 of the last pass: from the per-instance norms, or (pnorm) summed
  // here from the last update's chunk partials of this instance, in a fixed
  // order -- the update then needs no separate reduction launch
  {
    const bool ro0 = reorth && reorth[b] != 0;
    if (pnorm && (ro0 || !n1)) {
      // eight loads in flight per lane, summed in a fixed order
      const int c1 = kd.cptr[b + 1];
      double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int c = kd.cptr[b] + lane;
      for (; c + 7 * 64 < c1; c += 8 * 64) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += pnorm[c + u * 64];
      }
      for (; c < c1; c += 64) a[0] += pnorm[c];
      double t = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
      t = kwave_sum(t);
      if (lane == 0) s_nn = t;
    } else if (lane == 0) {
      s_nn = ro0 ? n2[b] : n1[b];
    }
  }
  double *H = kd.H + (int64_t)b * (m + 1) * m;
  double *cs = kd.cs + (int64_t)b * m, *sn = kd.sn + (int64_t)b * m, *g = kd.g + (int64_t)b * (m + 1);
  const bool ro = reorth && reorth[b] != 0;
  for (int i = lane; i <= j; i += 64)
    col[i] = s1[(int64_t)b * s1s + i] + (ro ? s2[(int64_t)b * s2s + i] : 0.0);
  for (int i = lane; i < j; i += 64) {
    c_s[i] = cs[i];
    s_s[i] = sn[i];
  }
  __syncthreads();
  if (lane == 0) {
    const double hn = sqrt(s_nn);
    double a = col[0];
    for (int i = 0; i < j; ++i) {
      const double nx = col[i + 1];
      col[i] = c_s[i] * a + s_s[i] * nx;
      a = -s_s[i] * a + c_s[i] * nx;
    }
    const double den = hypot(a, hn);
    const double c = den == 0.0 ? 1.0 : a / den;
    const double sj = den == 0.0 ? 0.0 : hn / den;
    cs[j] = c;
    sn[j] = sj;
    col[j] = c * a + sj * hn;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sj * gj;
    g[j] = c * gj;
    const int its = kd.its[b] + 1;
    kd.its[b] = its;
    const bool fin = !isfinite(hn) || !isfinite(g[j + 1]);
    if (fin) kd.status[b] = 2;
    if (fabs(g[j + 1]) <= kd.rtol[b] * kd.bnorm[b] || hn == 0.0 || its >= kd.itmax[b] || j + 1 == m || fin)
      kd.kconv[b] = j + 1;
    scale[b] = hn > 0.0 ? 1.0 / hn : 0.0;
  }
  __syncthreads();
  for (int i = lane; i <= j + 1; i += 64) H[i * m + j] = col[i];
}

// number of instances still iterating in this cycle -> *count
__global__ void k_count_active(KrylovDev kd, int *count) {
  __shared__ int sm[256];
  int c = 0;
  for (int b = threadIdx.x; b < kd.n_inst; b += 256) c += inst_on(kd, b) ? 1 : 0;
  sm[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = sm[0];
}

// y_b = H_b(1:k,1:k)^-1 g_b (back substitution), k = kconv[b]; est[b] = |g_b[k]|.
// One wavefront per instance: as each y_i becomes known its column is
// removed from the rows above it (in LDS; H staged in LDS when k <= 64).
constexpr int kSolveLds = 64;
__global__ __launch_bounds__(64) void k_solve_y(KrylovDev kd, int m, double *__restrict__ y,
                                                double *__restrict__ est) {
  __shared__ double Hs[kSolveLds][kSolveLds + 1];
  __shared__ double gs[kMaxKrylov + 1];
  const int b = blockIdx.x, lane = threadIdx.x;
  if (!kd.solving[b]) {  // uniform over the block
    if (lane == 0) kd.nbasis[b] = 0;
    return;
  }
  const int k = kd.kconv[b] < 0 ? m : kd.kconv[b];
  const double *H = kd.H + (int64_t)b * (m + 1) * m;
  const double *g = kd.g + (int64_t)b * (m + 1);
  for (int i = lane; i <= k; i += 64) gs[i] = g[i];
  if (k <= kSolveLds) {
    for (int t = lane; t < k * k; t += 64) {
      const int i = t / k, c = t % k;
      if (c >= i) Hs[i][c] = H[(int64_t)i * m + c];
    }
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
      const double yi = gs[i] / Hs[i][i];
      if (lane < i) gs[lane] -= Hs[lane][i] * yi;
      if (lane == 0) gs[i] = yi;
      __syncthreads();
    }
  } else {
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
      const double yi = gs[i] / H[(int64_t)i * m + i];
      for (int c = lane; c < i; c += 64) gs[c] -= H[(int64_t)c * m + i] * yi;
      if (lane == 0) gs[i] = yi;
      __syncthreads();
    }
  }
  double *yb = y + (int64_t)b * m;
  for (int i = lane; i < k; i += 64) yb[i] = gs[i];
  if (lane == 0) {
    kd.nbasis[b] = k;
    est[b] = fabs(g[k]);
  }
}

// start of a cycle: g = (beta, 0, ...), kconv = -1, scale = 1/beta for
// iterating instances with beta > 0 (an instance with beta = 0 is done)
__global__ void k_cycle_start(KrylovDev kd, int m, const double *__restrict__ beta2,
                              double *__restrict__ scale) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= kd.n_inst) return;
  double *g = kd.g + (int64_t)b * (m + 1);
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  kd.kconv[b] = -1;
  const double beta = sqrt(beta2[b]);
  g[0] = beta;
  scale[b] = (kd.solving[b] && beta > 0.0) ? 1.0 / beta : 0.0;
  if (kd.solving[b] && !(beta > 0.0)) kd.kconv[b] = 0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int RR>
static void sproj_launch(const KrylovDev &kd, const T *V, int64_t ldv, int k, const T *w,
                         const int *gate, double *partial, hipStream_t st) {
  hipLaunchKernelGGL((k_sproj<T, RR>), dim3(kd.n_chunks), dim3(kChunkRows / RR), 0, st, kd, V, ldv, k,
                     w, gate, partial);
}
template <typename T, int RR>
static void supdate_launch(const KrylovDev &kd, const T *V, int64_t ldv, int k, const double *h,
                           int hstride, T *w, const int *gate, double *partial, hipStream_t st) {
  hipLaunchKernelGGL((k_supdate<T, RR>), dim3(kd.n_chunks), dim3(kChunkRows / RR), 0, st, kd, V, ldv,
                     k, h, hstride, w, gate, partial);
}

template <typename T>
hipError_t ks_proj(const KrylovDev &kd, const T *V, int64_t ldv, int k, const T *w,
                   const int *gate, double *partial, double *out, hipStream_t st) {
  switch (kd.ortho_var) {
    case 1: sproj_launch<T, 8>(kd, V, ldv, k, w, gate, partial, st); break;
    case 2: sproj_launch<T, 2>(kd, V, ldv, k, w, gate, partial, st); break;
    default: sproj_launch<T, 4>(kd, V, ldv, k, w, gate, partial, st); break;
  }
  hipLaunchKernelGGL(k_seg_reduce, dim3(kd.n_inst, k + 1), dim3(KT), 0, st, kd, partial, k + 1, out);
  return hipGetLastError();
}
template <typename T>
hipError_t ks_update(const KrylovDev &kd, const T *V, int64_t ldv, int k, const double *h,
                     int hstride, T *w, const int *gate, double *partial, double *out,
                     hipStream_t st) {
  switch (kd.ortho_var) {
    case 1: supdate_launch<T, 8>(kd, V, ldv, k, h, hstride, w, gate, partial, st); break;
    case 2: supdate_launch<T, 2>(kd, V, ldv, k, h, hstride, w, gate, partial, st); break;
    default: supdate_launch<T, 4>(kd, V, ldv, k, h, hstride, w, gate, partial, st); break;
  }
  if (out) hipLaunchKernelGGL(k_seg_reduce, dim3(kd.n_inst, 1), dim3(KT), 0, st, kd, partial, 1, out);
  return hipGetLastError();
}
template <typename T>
hipError_t ks_scale(const KrylovDev &kd, const T *w, const double *scale, T *v, hipStream_t st) {
  hipLaunchKernelGGL(k_sscale<T>, dim3(kd.n_chunks), dim3(KT), 0, st, kd, w, scale, v);
  return hipGetLastError();
}
template <typename T>
hipError_t ks_combine(const KrylovDev &kd, const T *V, int64_t ldv, const double *y, int ystride,
                      T *out, hipStream_t st) {
  hipLaunchKernelGGL(k_scombine<T>, dim3(kd.n_chunks), dim3(KT), 0, st, kd, V, ldv, y, ystride,
                     kd.nbasis, out);
  return hipGetLastError();
}
template <typename TX, typename TZ>
hipError_t ks_axpy(const KrylovDev &kd, const double *coef, const TZ *z, TX *x, hipStream_t st) {
  hipLaunchKernelGGL((k_saxpy<TX, TZ>), dim3(kd.n_chunks), dim3(KT), 0, st, kd, coef, z, x);
  return hipGetLastError();
}
template <typename T>
hipError_t ks_sub(const KrylovDev &kd, const T *b, const T *jx, T *r, hipStream_t st) {
  hipLaunchKernelGGL(k_ssub<T>, dim3(kd.n_chunks), dim3(KT), 0, st, kd, b, jx, r);
  return hipGetLastError();
}
template <typename TY, typename TX>
hipError_t ks_cast(const KrylovDev &kd, const TX *x, const double *coef, TY *y, hipStream_t st) {
  hipLaunchKernelGGL((k_scast<TY, TX>), dim3(kd.n_chunks), dim3(KT), 0, st, kd, x, coef, y);
  return hipGetLastError();
}
hipError_t ks_copy(const KrylovDev &kd, const double *x, double *y, hipStream_t st) {
  hipLaunchKernelGGL(k_scopy<double>, dim3(kd.n_chunks), dim3(KT), 0, st, kd, x, y);
  return hipGetLastError();
}
template <typename T>
hipError_t ks_zero(const KrylovDev &kd, T *x, int only_solving, hipStream_t st) {
  hipLaunchKernelGGL(k_szero<T>, dim3(kd.n_chunks), dim3(KT), 0, st, kd, x, only_solving);
  return hipGetLastError();
}
template <typename T, int RR>
static void sproj2_launch(const KrylovDev &kd, const T *V, int64_t ldv, int k, const T *w,
                          double *partial, hipStream_t st) {
  hipLaunchKernelGGL((k_sproj2<T, RR>), dim3(kd.n_chunks), dim3(kChunkRows / RR), 0, st, kd, V, ldv, k,
                     w, partial);
}
template <typename T>
hipError_t ks_proj2(const KrylovDev &kd, const T *V, int64_t ldv, int k, const T *w, double *partial,
                    double *out, hipStream_t st) {
  switch (kd.ortho_var) {
    case 1: sproj2_launch<T, 8>(kd, V, ldv, k, w, partial, st); break;
    case 2: sproj2_launch<T, 2>(kd, V, ldv, k, w, partial, st); break;
    default: sproj2_launch<T, 4>(kd, V, ldv, k, w, partial, st); break;
  }
  hipLaunchKernelGGL(k_seg_reduce, dim3(kd.n_inst, 2 * k - 1), dim3(KT), 0, st, kd, partial, 2 * k - 1,
                     out);
  return hipGetLastError();
}
template hipError_t ks_proj2<double>(const KrylovDev &, const double *, int64_t, int, const double *,
                                     double *, double *, hipStream_t);
template hipError_t ks_proj2<float>(const KrylovDev &, const float *, int64_t, int, const float *,
                                    double *, double *, hipStream_t);
hipError_t ks_icwy(const KrylovDev &kd, int j, int m, const double *sv, double *Lmat, double *h,
                   int hstride, hipStream_t st) {
  hipLaunchKernelGGL(k_icwy, dim3(kd.n_inst), dim3(64), 0, st, kd, j, m, sv, Lmat, h, hstride);
  return hipGetLastError();
}

hipError_t ks_reorth_flag(const KrylovDev &kd, const double *n0, int n0s, const double *n1, int policy,
                          int *flag, hipStream_t st) {
  hipLaunchKernelGGL(k_reorth_flag, dim3((kd.n_inst + 63) / 64), dim3(64), 0, st, kd, n0, n0s, n1, policy,
                     flag);
  return hipGetLastError();
}
hipError_t ks_arnoldi(const KrylovDev &kd, int j, int m, const double *s1, int s1s, const double *s2,
                      int s2s, const int *reorth, const double *n1, const double *n2, const double *pnorm,
                      double *scale, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi, dim3(kd.n_inst), dim3(64), 0, st, kd, j, m, s1, s1s, s2, s2s, reorth,
                     n1, n2, pnorm, scale);
  return hipGetLastError();
}
hipError_t ks_count_active(const KrylovDev &kd, int *count, hipStream_t st) {
  hipLaunchKernelGGL(k_count_active, dim3(1), dim3(256), 0, st, kd, count);
  return hipGetLastError();
}
hipError_t ks_solve_y(const KrylovDev &kd, int m, double *y, double *est, hipStream_t st) {
  hipLaunchKernelGGL(k_solve_y, dim3(kd.n_inst), dim3(64), 0, st, kd, m, y, est);
  return hipGetLastError();
}
hipError_t ks_cycle_start(const KrylovDev &kd, int m, const double *beta2, double *scale,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_cycle_start, dim3((kd.n_inst + 63) / 64), dim3(64), 0, st, kd, m, beta2, scale);
  return hipGetLastError();
}

#define KS_INST(T)                                                                              \
  template hipError_t ks_proj<T>(const KrylovDev &, const T *, int64_t, int, const T *,          \
                                 const int *, double *, double *, hipStream_t);                 \
  template hipError_t ks_update<T>(const KrylovDev &, const T *, int64_t, int, const double *,   \
                                   int, T *, const int *, double *, double *, hipStream_t);     \
  template hipError_t ks_scale<T>(const KrylovDev &, const T *, const double *, T *, hipStream_t); \
  template hipError_t ks_combine<T>(const KrylovDev &, const T *, int64_t, const double *, int,  \
                                    T *, hipStream_t);                                          \
  template hipError_t ks_sub<T>(const KrylovDev &, const T *, const T *, T *, hipStream_t);      \
  template hipError_t ks_zero<T>(const KrylovDev &, T *, int, hipStream_t);
KS_INST(double)
KS_INST(float)
template hipError_t ks_axpy<double, double>(const KrylovDev &, const double *, const double *, double *, hipStream_t);
template hipError_t ks_axpy<float, float>(const KrylovDev &, const double *, const float *, float *, hipStream_t);
template hipError_t ks_axpy<double, float>(const KrylovDev &, const double *, const float *, double *, hipStream_t);
template hipError_t ks_cast<float, double>(const KrylovDev &, const double *, const double *, float *, hipStream_t);
template hipError_t ks_cast<double, double>(const KrylovDev &, const double *, const double *, double *, hipStream_t);


// ---------------------------------------------------------------------------
// per-instance norms and the Newton update (all instances, no gating)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(KT) void k_snorm2(KrylovDev kd, const T *__restrict__ x,
                                               double *__restrict__ partial) {
  __shared__ double wsum[KT / 64];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  double acc = 0.0;
  for (int rr = tid; rr < len; rr += KT) {
    const double v = (double)x[row0 + rr];
    acc += v * v;
  }
  acc = kwave_sum(acc);
  if (lane == 0) wsum[wv] = acc;
  __syncthreads();
  if (tid == 0) {
    double s2 = 0.0;
    for (int q = 0; q < KT / 64; ++q) s2 += wsum[q];
    partial[c] = s2;
  }
}

template <typename T>
hipError_t ks_norms(const KrylovDev &kd, const T *x, double *partial, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_snorm2<T>, dim3(kd.n_chunks), dim3(KT), 0, st, kd, x, partial);
  hipLaunchKernelGGL(k_seg_reduce, dim3(kd.n_inst, 1), dim3(KT), 0, st, kd, partial, 1, out);
  return hipGetLastError();
}
template hipError_t ks_norms<double>(const KrylovDev &, const double *, double *, double *, hipStream_t);
template hipError_t ks_norms<float>(const KrylovDev &, const float *, double *, double *, hipStream_t);

hipError_t launch_seg_norms(const KrylovDev &kd, const double *x, double *partial, double *out,
                            hipStream_t st) {
  return ks_norms<double>(kd, x, partial, out, st);
}

// partial[c*4 + (0..3)] = chunk sums of r^2 and b^2 on displacement rows
// (0, 1) and on pressure rows (2, 3); a chunk lies in one of the two parts
__global__ __launch_bounds__(KT) void k_snorm_up(KrylovDev kd, const double *__restrict__ r,
                                                 const double *__restrict__ bv, int64_t n_u,
                                                 double *__restrict__ partial) {
  __shared__ double wsum[2][KT / 64];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  double a0 = 0.0, a1 = 0.0;
  for (int rr = tid; rr < len; rr += KT) {
    const double x = r[row0 + rr], y = bv[row0 + rr];
    a0 += x * x;
    a1 += y * y;
  }
  a0 = kwave_sum(a0);
  a1 = kwave_sum(a1);
  if (lane == 0) {
    wsum[0][wv] = a0;
    wsum[1][wv] = a1;
  }
  __syncthreads();
  if (tid < 4) {
    const bool isp = row0 >= n_u;
    double s2 = 0.0;
    if ((tid >= 2) == isp)
      for (int q = 0; q < KT / 64; ++q) s2 += wsum[tid & 1][q];
    partial[(int64_t)c * 4 + tid] = s2;
  }
}

hipError_t launch_seg_norms_up(const KrylovDev &kd, const double *r, const double *b, int64_t n_u,
                               double *partial, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_snorm_up, dim3(kd.n_chunks), dim3(KT), 0, st, kd, r, b, n_u, partial);
  hipLaunchKernelGGL(k_seg_reduce, dim3(kd.n_inst, 4), dim3(KT), 0, st, kd, partial, 4, out);
  return hipGetLastError();
}

__global__ void k_begin(KrylovDev kd, const double *__restrict__ n2) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= kd.n_inst) return;
  kd.bnorm[b] = sqrt(n2[b]);
  kd.kconv[b] = -1;
  kd.its[b] = 0;
  kd.status[b] = 0;
}
hipError_t ks_begin(const KrylovDev &kd, const double *n2, hipStream_t st) {
  hipLaunchKernelGGL(k_begin, dim3((kd.n_inst + 63) / 64), dim3(64), 0, st, kd, n2);
  return hipGetLastError();
}

// x += dx on instances with upd[b] != 0 (p >= cut-off when enabled);
// partial[c*4 + (0..3)] = ||du||^2, ||u||^2, ||dp||^2, ||p||^2 of the chunk
__global__ __launch_bounds__(KT) void k_snewton_update(KrylovDev kd, const double *__restrict__ dx,
                                                       double *__restrict__ x, int64_t n_u,
                                                       const int *__restrict__ upd, int cutoff_on,
                                                       double cutoff, double *__restrict__ partial) {
  __shared__ double wsum[4][KT / 64];
  const int c = blockIdx.x, tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int b = kd.c_inst[c];
  const bool on = upd[b] != 0;
  const int64_t row0 = kd.c_row0[c];
  const int len = kd.c_len[c];
  double a0 = 0.0, a1 = 0.0;
  const bool isp = row0 >= n_u;
  for (int rr = tid; rr < len; rr += KT) {
    const int64_t r = row0 + rr;
    const double d = on ? dx[r] : 0.0;
    double v = x[r] + d;
    if (isp && on && cutoff_on && v < cutoff) v = cutoff;
    if (on) x[r] = v;
    a0 += d * d;
    a1 += v * v;
  }
  a0 = kwave_sum(a0);
  a1 = kwave_sum(a1);
  if (lane == 0) {
    wsum[isp ? 2 : 0][wv] = a0;
    wsum[isp ? 3 : 1][wv] = a1;
    wsum[isp ? 0 : 2][wv] = 0.0;
    wsum[isp ? 1 : 3][wv] = 0.0;
  }
  __syncthreads();
  if (tid < 4) {
    double s2 = 0.0;
    for (int q = 0; q < KT / 64; ++q) s2 += wsum[tid][q];
    partial[(int64_t)c * 4 + tid] = s2;
  }
}

hipError_t launch_snewton_update(const KrylovDev &kd, const double *dx, double *x, int64_t n_u,
                                 const int *upd, int cutoff_on, double cutoff, double *partial,
                                 double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_snewton_update, dim3(kd.n_chunks), dim3(KT), 0, st, kd, dx, x, n_u, upd,
                     cutoff_on, cutoff, partial);
  hipLaunchKernelGGL(k_seg_reduce, dim3(kd.n_inst, 4), dim3(KT), 0, st, kd, partial, 4, out);
  return hipGetLastError();
}

}  // namespace hf
