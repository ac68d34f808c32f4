// Two-level block preconditioner for gfx950: coarse space of P1 vertex
// classes (see hf_coarse.cpp), multifrontal Gauss-Jordan factorisation of
// the coarse matrix, and the kernels of one preconditioned product.
//
// Preconditioner (full block factorisation of J = [[A, B], [C, D]]):
//   A^-1 ~ Ah^-1 r = P z_c + M_A^-1 (r - A P z_c),  z_c = A_c^-1 P^T r,
//   A_c = P^T A P (the coarse matrix), M_A the element blocks,
//   S = D - C Ah^-1 B = (D - C M_A^-1 B) - W Z_c,  W = C P - (C M_A^-1) (A P),
//   Z_c = A_c^-1 P^T B;
//   z_p = S^-1 (v_p - C Ah^-1 v_u),  z_u = Ah^-1 (v_u - B z_p).
// The product w = J z the Krylov solver needs is formed without z:
//   q = C Ah^-1 v_u = Cf v_u + W z_c1,  z_c1 = A_c^-1 P^T v_u,
//   z_p = S^-1 (v_p - q),
//   z_c2 = A_c^-1 P^T (v_u - B z_p) = z_c1 - Z_c z_p,
//   t = v_u - B z_p - A P z_c2,
//   w_u = Af t + B z_p + A P z_c2,  w_p = v_p,
// with Af = A M_A^-1 and Cf = C M_A^-1 the folded blocks: the factorisation
// M differs from J only in its displacement block (Ah for A), so the
// pressure rows of J M^-1 are those of the identity.
//
// Front layout: row-major f x f; the first k rows / columns are the node's
// own DOFs.  After the elimination a front holds
//   [[F11^-1, F11^-1 F12], [-F21 F11^-1, F22 - F21 F11^-1 F12]].
#include <algorithm>
#include <cmath>

#include "hf_internal.h"

namespace hf {

constexpr int kCT = 256;   // threads of the row-parallel kernels
constexpr int kNB = 32;    // Gauss-Jordan panel width
constexpr int kTile = 64;  // tile of the Gauss-Jordan update

__device__ inline bool clamped(const uint32_t *clamp, int64_t e, int r) { return (clamp[e] >> r) & 1u; }

// ---------------------------------------------------------------------------
// A P panels: AP_e (bu x ncol*dim, column-major) = sum over the blocks of
// row e of A_ef P_f.  One workgroup per element row, one thread per entry.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCT) void k_ap_build(KParams kp, CoarseK ck, const double *__restrict__ A,
                                                  const int32_t *__restrict__ elist, double *__restrict__ AP) {
  const int64_t e = elist ? elist[blockIdx.x] : blockIdx.x;
  const int bu = kp.s.bu, dim = ck.dim, nv = ck.nv;
  const int64_t c0 = ck.ap_ptr[e];
  const int ncol = (int)(ck.ap_ptr[e + 1] - c0);
  const int64_t b0 = kp.m.blk_ptr[e], b1 = kp.m.blk_ptr[e + 1];
  double *out = AP + c0 * dim * bu;
  for (int t = threadIdx.x; t < ncol * dim * bu; t += kCT) {
    const int r = t % bu, col = t / bu, j = col / dim, k = col % dim;
    const int32_t cls = ck.ap_cls[c0 + j];
    double acc = 0.0;
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t f = kp.m.blk_col[b];
      const double *Ab = A + b * bu * bu;
      for (int v = 0; v < nv; ++v) {
        if (ck.cls_of[f * nv + v] != cls) continue;
        for (int q = 0; q < ck.nw[v]; ++q) {
          const int a = ck.wn[v][q];
          if (clamped(kp.m.clamp, f, a * dim + k)) continue;
          acc += ck.ww[v][q] * Ab[(int64_t)(a * dim + k) * bu + r];
        }
      }
    }
    out[t] = acc;
  }
}

// W rows per strip entry: W_ent = C_ent P_e - (C_ent M_e^-1) AP_e over the
// AP columns of the entry's element (one workgroup per strip entry)
__global__ __launch_bounds__(kCT) void k_w_build(KParams kp, CoarseK ck, const double *__restrict__ Cs,
                                                 const double *__restrict__ inv, const double *__restrict__ AP,
                                                 double *__restrict__ W) {
  const int64_t ent = blockIdx.x;
  const int bu = kp.s.bu, dim = ck.dim, nv = ck.nv;
  const int64_t e = kp.m.sp_elem[ent];
  const int64_t c0 = ck.ap_ptr[e];
  const int ncol = (int)(ck.ap_ptr[e + 1] - c0);
  __shared__ double cf[32];
  const double *Ce = Cs + ent * bu;
  const double *ie = inv + e * bu * bu;
  for (int r = threadIdx.x; r < bu; r += kCT) {
    double acc = 0.0;
    for (int s = 0; s < bu; ++s) acc += Ce[s] * ie[(int64_t)r * bu + s];
    cf[r] = acc;
  }
  __syncthreads();
  const double *ap = AP + c0 * dim * bu;
  double *out = W + ck.w_off[ent];
  for (int col = threadIdx.x; col < ncol * dim; col += kCT) {
    const int j = col / dim, k = col % dim;
    const int32_t cls = ck.ap_cls[c0 + j];
    double acc = 0.0;
    for (int v = 0; v < nv; ++v) {
      if (ck.cls_of[e * nv + v] != cls) continue;
      for (int q = 0; q < ck.nw[v]; ++q) {
        const int a = ck.wn[v][q];
        if (!clamped(kp.m.clamp, e, a * dim + k)) acc += ck.ww[v][q] * Ce[a * dim + k];
      }
    }
    for (int r = 0; r < bu; ++r) acc -= cf[r] * ap[(int64_t)col * bu + r];
    out[col] = acc;
  }
}

// coarse matrix entries into the fronts: thread per (pair, i, k)
__global__ __launch_bounds__(kCT) void k_pairs(KParams kp, CoarseK ck, const double *__restrict__ AP,
                                               double *__restrict__ F) {
  const int dim = ck.dim, d2 = dim * dim, bu = kp.s.bu, nv = ck.nv;
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= ck.n_pairs * d2) return;
  const int64_t p = t / d2;
  const int i = (int)(t % d2) / dim, k = (int)(t % d2) % dim;
  double acc = 0.0;
  for (int64_t c = ck.pair_cptr[p]; c < ck.pair_cptr[p + 1]; ++c) {
    const int64_t e = ck.pc_e[c];
    const int v = ck.pc_vj[c] & 255, j = ck.pc_vj[c] >> 8;
    const double *ap = AP + ck.ap_ptr[e] * dim * bu + (int64_t)(j * dim + k) * bu;
    for (int q = 0; q < ck.nw[v]; ++q) {
      const int a = ck.wn[v][q];
      if (!clamped(kp.m.clamp, e, a * dim + i)) acc += ck.ww[v][q] * ap[a * dim + i];
    }
  }
  (void)nv;
  F[ck.pair_dest[p] + (int64_t)i * ck.pair_ld[p] + k] = acc;
}

__global__ void k_cfill(double *__restrict__ x, int64_t n) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    x[t] = 0.0;
}

// extend-add of the update blocks of the children in one slot into the
// fronts of the parents at level lev (grid: entry tiles x parents)
__global__ __launch_bounds__(kCT) void k_extend_add(CoarseK ck, int lev, int slot, double *__restrict__ F) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int ch = ck.children[2 * x + slot];
  if (ch < 0) return;
  const int dim = ck.dim;
  const int fc = ck.ff[ch], kc = ck.fk[ch], m = fc - kc;
  const int fp = ck.ff[x];
  const int64_t n = (int64_t)m * m;
  const int32_t *map = ck.ea_map + ck.ea_ptr[ch];
  const double *src = F + ck.fo[ch];
  double *dst = F + ck.fo[x];
  for (int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x; t < n; t += (int64_t)gridDim.x * kCT) {
    const int a = (int)(t / m), b = (int)(t % m);
    const int pa = map[a / dim] * dim + a % dim, pb = map[b / dim] * dim + b % dim;
    dst[(int64_t)pa * fp + pb] += src[(int64_t)(kc + a) * fc + kc + b];
  }
}

// ---------------------------------------------------------------------------
// Multifrontal Gauss-Jordan, one panel of kNB pivots [p0, p0 + nb) of every
// front at a level whose k exceeds p0.
// Kernel A: invert the panel's diagonal block D (in LDS, no pivoting: the
// coarse matrix is a stiffness), scale the row panel F[K, j] <- D^-1 F[K, j]
// (j outside K), keep a copy of the column panel and D^-1 for kernel B.
// ---------------------------------------------------------------------------
__device__ bool panel_inverse(const double *F, int f, int p0, int nb, double (*D)[kNB + 1]) {
  for (int t = threadIdx.x; t < nb * nb; t += kCT) D[t / nb][t % nb] = F[(int64_t)(p0 + t / nb) * f + p0 + t % nb];
  __syncthreads();
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const double pv = D[k][k];
    const bool ok = fabs(pv) > 0.0 && isfinite(pv);
    if (!ok) {
      if (threadIdx.x == 0) bad = 1;
      __syncthreads();
      return false;
    }
    const double pinv = 1.0 / pv;
    __syncthreads();
    if ((int)threadIdx.x < nb) D[k][threadIdx.x] = (int)threadIdx.x == k ? pinv : D[k][threadIdx.x] * pinv;
    __syncthreads();
    double fk[(kNB * kNB + kCT - 1) / kCT];
    int cnt = 0;
    for (int t = threadIdx.x; t < nb * nb; t += kCT) fk[cnt++] = D[t / nb][k];
    __syncthreads();
    cnt = 0;
    for (int t = threadIdx.x; t < nb * nb; t += kCT) {
      const int r = t / nb, c = t % nb;
      const double fr = fk[cnt++];
      if (r != k) D[r][c] = c == k ? -fr * pinv : D[r][c] - fr * D[k][c];
    }
    __syncthreads();
  }
  return bad == 0;
}

__global__ __launch_bounds__(kCT) void k_gj_a(CoarseK ck, int lev, int p0, double *__restrict__ F,
                                              double *__restrict__ Cp, double *__restrict__ Dsc, int *flag) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  if (p0 >= k) return;
  const int nb = min(kNB, k - p0);
  const int tile = blockIdx.x;
  if (tile * kTile >= f) return;
  double *Fx = F + ck.fo[x];
  __shared__ double D[kNB][kNB + 1];
  if (!panel_inverse(Fx, f, p0, nb, D)) {
    if (threadIdx.x == 0) atomicOr(flag, 1);
    return;
  }
  // rows [tile*64, +64) of the column panel, before kernel B changes it
  double *cp = Cp + ck.cpo[x];
  for (int t = threadIdx.x; t < kTile * nb; t += kCT) {
    const int r = tile * kTile + t / nb, c = t % nb;
    if (r < f) cp[(int64_t)r * kNB + c] = Fx[(int64_t)r * f + p0 + c];
  }
  if (tile == 0)
    for (int t = threadIdx.x; t < nb * nb; t += kCT) Dsc[(int64_t)blockIdx.y * kNB * kNB + t] = D[t / nb][t % nb];
  // columns [tile*64, +64) of the row panel: F[K, j] <- D^-1 F[K, j]
  __shared__ double R[kNB][kTile];
  for (int t = threadIdx.x; t < nb * kTile; t += kCT) {
    const int r = t / kTile, c = tile * kTile + t % kTile;
    R[r][t % kTile] = c < f ? Fx[(int64_t)(p0 + r) * f + c] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * kTile; t += kCT) {
    const int r = t / kTile, cl = t % kTile, c = tile * kTile + cl;
    if (c >= f || (c >= p0 && c < p0 + nb)) continue;
    double acc = 0.0;
    for (int s = 0; s < nb; ++s) acc += D[r][s] * R[s][cl];
    Fx[(int64_t)(p0 + r) * f + c] = acc;
  }
}

// Kernel B: F[i, j] -= Cp[i, :] F[K, j] outside the panel rows and columns,
// F[i, K] = -Cp[i, :] D^-1 outside the panel rows, F[K, K] = D^-1
__global__ __launch_bounds__(kCT) void k_gj_b(CoarseK ck, int lev, int p0, double *__restrict__ F,
                                              const double *__restrict__ Cp, const double *__restrict__ Dsc,
                                              const int *flag) {
  if (*flag) return;
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  if (p0 >= k) return;
  const int nb = min(kNB, k - p0);
  const int nt = (f + kTile - 1) / kTile;
  const int ti = blockIdx.x / nt, tj = blockIdx.x % nt;
  if (ti >= nt) return;
  double *Fx = F + ck.fo[x];
  const double *cp = Cp + ck.cpo[x];
  const double *Dn = Dsc + (int64_t)blockIdx.y * kNB * kNB;
  __shared__ double Ct[kTile][kNB + 1];
  __shared__ double Rt[kNB][kTile + 1];
  __shared__ double Dt[kNB][kNB + 1];
  const int i0 = ti * kTile, j0 = tj * kTile;
  for (int t = threadIdx.x; t < kTile * kNB; t += kCT) {
    const int r = t / kNB, c = t % kNB;
    Ct[r][c] = (i0 + r < f && c < nb) ? cp[(int64_t)(i0 + r) * kNB + c] : 0.0;
  }
  for (int t = threadIdx.x; t < kNB * kTile; t += kCT) {
    const int r = t / kTile, c = t % kTile;
    Rt[r][c] = (r < nb && j0 + c < f) ? Fx[(int64_t)(p0 + r) * f + j0 + c] : 0.0;
  }
  for (int t = threadIdx.x; t < kNB * kNB; t += kCT) {
    const int r = t / kNB, c = t % kNB;
    Dt[r][c] = (r < nb && c < nb) ? Dn[r * nb + c] : 0.0;
  }
  __syncthreads();
  // 4 x 4 entries per thread
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int il = tr * 4 + a, i = i0 + il;
    if (i >= f) continue;
    const bool iK = i >= p0 && i < p0 + nb;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int jl = tc + 16 * b, j = j0 + jl;
      if (j >= f) continue;
      const bool jK = j >= p0 && j < p0 + nb;
      if (iK && !jK) continue;  // the row panel, done by kernel A
      double *dst = Fx + (int64_t)i * f + j;
      if (iK && jK) {
        *dst = Dt[i - p0][j - p0];
      } else if (jK) {
        double acc = 0.0;
        for (int s = 0; s < nb; ++s) acc += Ct[il][s] * Dt[s][j - p0];
        *dst = -acc;
      } else {
        double acc = 0.0;
        for (int s = 0; s < nb; ++s) acc += Ct[il][s] * Rt[s][jl];
        *dst -= acc;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Dense P^T B (coarse rows x the pressure columns of each instance,
// row-major with nrhs columns): thread per (class, component)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCT) void k_ptb(KParams kp, CoarseK ck, const double *__restrict__ Bs, int nrhs,
                                             double *__restrict__ R) {
  const int dim = ck.dim, nv = ck.nv, bu = kp.s.bu;
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= (int64_t)ck.ncls * dim) return;
  const int32_t c = (int32_t)(t / dim);
  const int i = (int)(t % dim);
  double *row = R + t * nrhs;
  for (int j = 0; j < nrhs; ++j) row[j] = 0.0;
  const int b = ck.cinst[c];
  const int32_t p0 = kp.poff[b];
  for (int32_t q = ck.rc_ptr[c]; q < ck.rc_ptr[c + 1]; ++q) {
    const int64_t e = ck.rc_list[q] / nv;
    const int v = ck.rc_list[q] % nv;
    for (int64_t s = kp.m.sp_ptr[e]; s < kp.m.sp_ptr[e + 1]; ++s) {
      double acc = 0.0;
      for (int w = 0; w < ck.nw[v]; ++w) {
        const int a = ck.wn[v][w];
        if (!clamped(kp.m.clamp, e, a * dim + i)) acc += ck.ww[v][w] * Bs[s * bu + a * dim + i];
      }
      row[kp.m.sp_pnode[s] - p0] += acc;
    }
  }
}

// S_b[i][j] -= sum over i's strip entries of W_ent . Z_c[:, j] (the pressure
// block of each instance; Z_c row-major with nrhs columns)
__global__ __launch_bounds__(kCT) void k_s_correct(KParams kp, CoarseK ck, const double *__restrict__ W,
                                                   const double *__restrict__ Z, int nrhs, double *__restrict__ S) {
  const int64_t i = blockIdx.y;
  const int b = kp.pinst[i];
  const int64_t p0 = kp.poff[b], nb = kp.poff[b + 1] - p0;
  const int64_t j = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (j >= nb) return;
  const int dim = ck.dim;
  double acc = 0.0;
  for (int32_t c = kp.m.pc_ptr[i]; c < kp.m.pc_ptr[i + 1]; ++c) {
    const int32_t ent = kp.m.pc_ent[c];
    const int64_t e = kp.m.sp_elem[ent];
    const int64_t c0 = ck.ap_ptr[e];
    const int ncol = (int)(ck.ap_ptr[e + 1] - c0);
    const double *w = W + ck.w_off[ent];
    for (int col = 0; col < ncol * dim; ++col)
      acc += w[col] * Z[((int64_t)ck.ap_cls[c0 + col / dim] * dim + col % dim) * nrhs + j];
  }
  S[kp.doff[b] + (i - p0) * nb + j] -= acc;
}

// ---------------------------------------------------------------------------
// Coarse solves.  Forward, level by level from the leaves: the node's own
// right-hand side v = b_own + the children's update rows at its own
// positions is kept in y; the update rows of its struct positions are
// u = (children's rows there) + (-F21 F11^-1) v.  Backward, from the root:
// x_own = F11^-1 v - (F11^-1 F12) x_struct.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T own_rhs(const CoarseK &ck, int64_t pos, const T *b, const T *upd, int nrhs, int j) {
  T v = b[(int64_t)ck.fd_dof[pos] * nrhs + j];
  if (ck.src0[pos] >= 0) v += upd[ck.src0[pos] * nrhs + j];
  if (ck.src1[pos] >= 0) v += upd[ck.src1[pos] * nrhs + j];
  return v;
}

// one right-hand side.  Forward: each own position's right-hand side is
// formed once (one thread each) into y and into the front vector cv, then
// one wavefront per struct row reads its row of the column panel against
// cv.  Backward: the front vector [y_own; -x_struct] is gathered once, then
// one wavefront per own row reads its row of [F11^-1, F11^-1 F12].  The
// front vectors are contiguous, so the rows stream without index loads.
template <typename T>
__global__ __launch_bounds__(kCT) void k_fwd_own(CoarseK ck, int lev, const T *__restrict__ b,
                                                 const T *__restrict__ upd, T *__restrict__ y, T *__restrict__ cv) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int c = blockIdx.x * kCT + threadIdx.x;
  if (c >= ck.fk[x]) return;
  const int64_t pos = ck.fd_ptr[x] + c;
  const T v = own_rhs<T>(ck, pos, b, upd, 1, 0);
  y[ck.fd_dof[pos]] = v;
  cv[pos] = v;
}

// Lanes per row of a front's row products: short rows take a segment of a
// wave (16 or 32 lanes, two or four rows per wave) so that the lanes stay
// busy; the choice depends on the front alone, so a front is summed the same
// way in a batch and alone.
__host__ __device__ inline int row_lanes(int len) { return len <= 256 ? 16 : (len <= 1024 ? 32 : 64); }

// dot product of one row segment with the front vector; the lanes of a
// segment reduce among themselves (segments are aligned, so every lane of a
// segment has the same row and either all of them or none return early).
// LONG (levels whose rows exceed kLongRow entries, near the root): a lane
// first takes its entries in whole chunks of kDotChunk whose loads are issued
// together, since such a row is otherwise a chain of dependent HBM round
// trips; the rest goes one at a time.  The chunks cost registers, so the
// levels of short rows (the leaves) keep the plain loop.  Each lane adds its
// products in the same order, one fused multiply-add each, either way, so a
// front's result does not depend on the path its level takes (in a batch the
// longest row of the level over all instances picks it).
constexpr int kLongRow = 1024;
constexpr int kDotChunk = 16;
template <typename T, typename TF, bool LONG = false>
__device__ inline double row_dot(const TF *__restrict__ row, const T *__restrict__ v, int len, int sl, int lpr) {
  double acc = 0.0;
  int c = sl;
  if constexpr (LONG) {
    for (; c + (kDotChunk - 1) * lpr < len; c += kDotChunk * lpr) {
      TF x[kDotChunk];
      double y[kDotChunk];
#pragma unroll
      for (int u = 0; u < kDotChunk; ++u) {
        x[u] = __builtin_nontemporal_load(row + c + u * lpr);
        y[u] = (double)v[c + u * lpr];
      }
#pragma unroll
      for (int u = 0; u < kDotChunk; ++u) acc += (double)x[u] * y[u];
    }
  }
#pragma unroll 4
  for (; c < len; c += lpr) acc += (double)__builtin_nontemporal_load(row + c) * (double)v[c];
  for (int off = lpr / 2; off > 0; off >>= 1) acc += __shfl_down(acc, off, lpr);
  return acc;
}

template <typename T, typename TF, bool LONG>
__global__ __launch_bounds__(kCT) void k_fwd_rows(CoarseK ck, int lev, const TF *__restrict__ Fm,
                                                  const T *__restrict__ cv, T *__restrict__ upd) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  const int lpr = row_lanes(k), rpb = kCT / lpr;  // lanes per row, rows per workgroup pass
  const int sl = threadIdx.x % lpr;
  const int64_t fd = ck.fd_ptr[x];
  // the workgroups of a front stride over its rows (the grid is sized for the
  // level's longest rows, so fronts with short rows need fewer passes)
  for (int r = k + blockIdx.x * rpb + threadIdx.x / lpr; r < f; r += gridDim.x * rpb) {
    double acc = row_dot<T, TF, LONG>(Fm + ck.fo[x] + (int64_t)r * f, cv + fd, k, sl, lpr);
    if (sl == 0) {
      const int64_t pos = fd + r;
      if (ck.src0[pos] >= 0) acc += (double)upd[ck.src0[pos]];
      if (ck.src1[pos] >= 0) acc += (double)upd[ck.src1[pos]];
      upd[ck.uo[x] + r - k] = (T)acc;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kCT) void k_bwd_gather(CoarseK ck, int lev, const T *__restrict__ y,
                                                    const T *__restrict__ xs, T *__restrict__ cv) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int c = blockIdx.x * kCT + threadIdx.x;
  if (c >= ck.ff[x]) return;
  const int64_t pos = ck.fd_ptr[x] + c;
  cv[pos] = c < ck.fk[x] ? y[ck.fd_dof[pos]] : -xs[ck.fd_dof[pos]];
}

template <typename T, typename TF, bool LONG>
__global__ __launch_bounds__(kCT) void k_bwd_rows(CoarseK ck, int lev, const TF *__restrict__ Fm,
                                                  const T *__restrict__ cv, T *__restrict__ xs) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  const int lpr = row_lanes(f), rpb = kCT / lpr;
  const int sl = threadIdx.x % lpr;
  const int64_t fd = ck.fd_ptr[x];
  for (int r = blockIdx.x * rpb + threadIdx.x / lpr; r < k; r += gridDim.x * rpb) {
    const double acc = row_dot<T, TF, LONG>(Fm + ck.fo[x] + (int64_t)r * f, cv + fd, f, sl, lpr);
    if (sl == 0) xs[ck.fd_dof[fd + r]] = (T)acc;
  }
}

// The same two sweeps with the front vector staged in LDS by every workgroup
// of the front (levels whose fronts hold at most kFrontLds values and take
// at most kFusedMaxGroups workgroups): the
// forward kernel forms the own right-hand sides itself (workgroup 0 also
// stores them in y) and the backward one gathers [y_own; -x_struct] itself,
// so each level takes one launch instead of two.  The products read the same
// values in the same order as with the staged front vector in memory.
constexpr int kFrontLds = 2048;
// every workgroup of a front stages the whole front vector, so the fused form
// is used only where a front takes few workgroups (measured: with up to ~125
// per front the redundant gathers cost more than the saved launches)
constexpr unsigned kFusedMaxGroups = 8;

template <typename T>
__device__ inline double row_dot_lds(const T *__restrict__ row, const double *__restrict__ v, int len, int sl,
                                     int lpr) {
  double acc = 0.0;
#pragma unroll 4
  for (int c = sl; c < len; c += lpr) acc += (double)__builtin_nontemporal_load(row + c) * v[c];
  for (int off = lpr / 2; off > 0; off >>= 1) acc += __shfl_down(acc, off, lpr);
  return acc;
}

template <typename T, typename TF>
__global__ __launch_bounds__(kCT) void k_fwd_fused(CoarseK ck, int lev, const TF *__restrict__ Fm,
                                                   const T *__restrict__ b, T *__restrict__ upd,
                                                   T *__restrict__ y) {
  __shared__ double sv[kFrontLds];
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  const int64_t fd = ck.fd_ptr[x];
  for (int c = threadIdx.x; c < k; c += kCT) {
    const T v = own_rhs<T>(ck, fd + c, b, upd, 1, 0);
    sv[c] = (double)v;
    if (blockIdx.x == 0) y[ck.fd_dof[fd + c]] = v;
  }
  __syncthreads();
  const int lpr = row_lanes(k), rpb = kCT / lpr;
  const int sl = threadIdx.x % lpr;
  for (int r = k + blockIdx.x * rpb + threadIdx.x / lpr; r < f; r += gridDim.x * rpb) {
    double acc = row_dot_lds<TF>(Fm + ck.fo[x] + (int64_t)r * f, sv, k, sl, lpr);
    if (sl == 0) {
      const int64_t pos = fd + r;
      if (ck.src0[pos] >= 0) acc += (double)upd[ck.src0[pos]];
      if (ck.src1[pos] >= 0) acc += (double)upd[ck.src1[pos]];
      upd[ck.uo[x] + r - k] = (T)acc;
    }
  }
}

template <typename T, typename TF>
__global__ __launch_bounds__(kCT) void k_bwd_fused(CoarseK ck, int lev, const TF *__restrict__ Fm,
                                                   const T *__restrict__ y, T *__restrict__ xs) {
  __shared__ double sv[kFrontLds];
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  const int64_t fd = ck.fd_ptr[x];
  for (int c = threadIdx.x; c < f; c += kCT) {
    const T v = c < k ? y[ck.fd_dof[fd + c]] : -xs[ck.fd_dof[fd + c]];
    sv[c] = (double)v;
  }
  __syncthreads();
  const int lpr = row_lanes(f), rpb = kCT / lpr;
  const int sl = threadIdx.x % lpr;
  for (int r = blockIdx.x * rpb + threadIdx.x / lpr; r < k; r += gridDim.x * rpb) {
    const double acc = row_dot_lds<TF>(Fm + ck.fo[x] + (int64_t)r * f, sv, f, sl, lpr);
    if (sl == 0) xs[ck.fd_dof[fd + r]] = (T)acc;
  }
}

// several right-hand sides (row-major, nrhs columns): own rows first, then
// the struct rows, a thread per (row, column)
__global__ __launch_bounds__(kCT) void k_fwdm_own(CoarseK ck, int lev, const double *__restrict__ b,
                                                  const double *__restrict__ upd, int nrhs, double *__restrict__ y) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x];
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= (int64_t)k * nrhs) return;
  const int r = (int)(t / nrhs), j = (int)(t % nrhs);
  const int64_t pos = ck.fd_ptr[x] + r;
  y[(int64_t)ck.fd_dof[pos] * nrhs + j] = own_rhs<double>(ck, pos, b, upd, nrhs, j);
}

template <typename TF>
__global__ __launch_bounds__(kCT) void k_fwdm_upd(CoarseK ck, int lev, const TF *__restrict__ Fm,
                                                  const double *__restrict__ y, int nrhs, double *upd) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= (int64_t)(f - k) * nrhs) return;
  const int r = k + (int)(t / nrhs), j = (int)(t % nrhs);
  const int64_t fd = ck.fd_ptr[x], pos = fd + r;
  const TF *row = Fm + ck.fo[x] + (int64_t)r * f;
  double acc = 0.0;
  for (int c = 0; c < k; ++c) acc += (double)row[c] * y[(int64_t)ck.fd_dof[fd + c] * nrhs + j];
  if (ck.src0[pos] >= 0) acc += upd[ck.src0[pos] * nrhs + j];
  if (ck.src1[pos] >= 0) acc += upd[ck.src1[pos] * nrhs + j];
  // the children's rows read here belong to lower levels (earlier launches)
  upd[(ck.uo[x] + r - k) * nrhs + j] = acc;
}

template <typename TF>
__global__ __launch_bounds__(kCT) void k_bwdm(CoarseK ck, int lev, const TF *__restrict__ Fm,
                                              const double *__restrict__ y, int nrhs, double *__restrict__ xs) {
  const int x = ck.level_nodes[ck.level_ptr[lev] + blockIdx.y];
  const int k = ck.fk[x], f = ck.ff[x];
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= (int64_t)k * nrhs) return;
  const int r = (int)(t / nrhs), j = (int)(t % nrhs);
  const int64_t fd = ck.fd_ptr[x];
  const TF *row = Fm + ck.fo[x] + (int64_t)r * f;
  double acc = 0.0;
  for (int c = 0; c < k; ++c) acc += (double)row[c] * y[(int64_t)ck.fd_dof[fd + c] * nrhs + j];
  for (int c = k; c < f; ++c) acc -= (double)row[c] * xs[(int64_t)ck.fd_dof[fd + c] * nrhs + j];
  xs[(int64_t)ck.fd_dof[fd + r] * nrhs + j] = acc;
}

// ---------------------------------------------------------------------------
// Kernels of one preconditioned product (precision T)
// ---------------------------------------------------------------------------
// P_e^T v_e per vertex copy: cpy[(e*nv + v)*dim + i] (thread per entry)
template <typename T>
__global__ __launch_bounds__(kCT) void k_restrict_copies(KParams kp, CoarseK ck, const T *__restrict__ v,
                                                         T *__restrict__ cpy) {
  const int dim = ck.dim, nv = ck.nv, nn = ck.nn;
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= kp.s.ne * nv * dim) return;
  const int64_t e = t / (nv * dim);
  const int vv = (int)(t / dim % nv), i = (int)(t % dim);
  double acc = 0.0;
  for (int w = 0; w < ck.nw[vv]; ++w) {
    const int a = ck.wn[vv][w];
    if (!clamped(kp.m.clamp, e, a * dim + i)) acc += ck.ww[vv][w] * (double)v[(e * nn + a) * dim + i];
  }
  cpy[t] = (T)acc;
}

// rc = sum over the copies of each class (thread per (class, component))
template <typename T>
__global__ __launch_bounds__(kCT) void k_restrict_gather(CoarseK ck, const T *__restrict__ cpy, T *__restrict__ rc) {
  const int dim = ck.dim;
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= (int64_t)ck.ncls * dim) return;
  const int32_t c = (int32_t)(t / dim);
  const int i = (int)(t % dim);
  double acc = 0.0;
  for (int32_t q = ck.rc_ptr[c]; q < ck.rc_ptr[c + 1]; ++q) acc += (double)cpy[(int64_t)ck.rc_list[q] * dim + i];
  rc[t] = (T)acc;
}

// z_c2 = z_c1 - Z_c z_p (Z_c row-major, nrhs columns: the pressure nodes of
// the row's instance); one wavefront per coarse DOF
template <typename T>
__global__ __launch_bounds__(kCT) void k_zc2(KParams kp, CoarseK ck, const T *__restrict__ Z, int nrhs,
                                             const T *__restrict__ zc1, const T *__restrict__ zp,
                                             T *__restrict__ zc2) {
  // a 16-lane segment of a wave per row (rows are as long as the instance's
  // pressure unknowns, a few hundred: a whole wave would leave most lanes idle)
  constexpr int LPR = 16;
  const int64_t r = (blockIdx.x * (int64_t)kCT + threadIdx.x) / LPR;
  const int sl = threadIdx.x % LPR;
  if (r >= (int64_t)ck.ncls * ck.dim) return;
  const int b = ck.cinst[r / ck.dim];
  const int32_t p0 = kp.poff[b], np = kp.poff[b + 1] - p0;
  const double acc = row_dot<T, T>(Z + r * nrhs, zp + p0, np, sl, LPR);
  if (sl == 0) zc2[r] = (T)((double)zc1[r] - acc);
}

// pressure rows of the first half: q'_i = v_p,i - (Cf v_u + W z_c1)_i
template <typename T>
__global__ __launch_bounds__(64) void k_tl_q(KParams kp, CoarseK ck, const T *__restrict__ Cf,
                                             const T *__restrict__ W, const T *__restrict__ vu,
                                             const T *__restrict__ vp, const T *__restrict__ zc,
                                             T *__restrict__ qout, T *__restrict__ wp) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x, bu = kp.s.bu, dim = ck.dim;
  double acc = 0.0;
  for (int32_t c = kp.m.pc_ptr[i]; c < kp.m.pc_ptr[i + 1]; ++c) {
    const int32_t ent = kp.m.pc_ent[c];
    const int64_t e = kp.m.sp_elem[ent];
    if (lane < bu) acc += (double)Cf[(int64_t)ent * bu + lane] * (double)vu[e * bu + lane];
    const int64_t c0 = ck.ap_ptr[e];
    const int ncol = (int)(ck.ap_ptr[e + 1] - c0) * dim;
    const T *w = W + ck.w_off[ent];
    for (int col = lane; col < ncol; col += 64)
      acc += (double)w[col] * (double)zc[(int64_t)ck.ap_cls[c0 + col / dim] * dim + col % dim];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    qout[i] = (T)((double)vp[i] - acc);
    if (wp) wp[i] = vp[i];
  }
}

// t = v_u - B z_p - AP z_c2 and apz = AP z_c2: thread per (element, row)
// columns of one element row of A P whose coarse values a workgroup stages in
// LDS (an element touches at most 20 vertex classes: 60 columns in 3D, 24 in 2D)
constexpr int kTlCols = 64;

template <typename T>
struct Pair;
template <>
struct Pair<double> {
  using type = double2;
};
template <>
struct Pair<float> {
  using type = float2;
};

// t = v_u - B z_p - AP z_c2 and apz = AP z_c2, one thread per pair of rows
// (2j, 2j+1) of an element row (block sizes are even), reading both rows'
// entries of a column of A P with one two-wide load
template <typename T>
__global__ __launch_bounds__(kCT) void k_tl_t(KParams kp, CoarseK ck, const T *__restrict__ AP,
                                              const T *__restrict__ Bs, const T *__restrict__ vu,
                                              const T *__restrict__ zp, const T *__restrict__ zc,
                                              T *__restrict__ t_out, T *__restrict__ apz) {
  using V2 = typename Pair<T>::type;
  // the workgroup's elements (at most tl_t_elems(bu)) get their z_c values
  // staged once in dynamic LDS sized for the block size, so the row loop
  // streams A P alone (a 30 x 30 block size needs 9.7 KB, not the 44.5 KB of
  // the 6 x 6 case, which leaves room for more resident workgroups)
  extern __shared__ double zs[];
  const int bu = kp.s.bu, hb = bu / 2, dim = ck.dim;
  const int64_t npair = kp.s.n_u / 2;
  const int64_t q0 = blockIdx.x * (int64_t)kCT;
  const int64_t e0 = q0 / hb;
  const int64_t e1 = (std::min<int64_t>(q0 + kCT, npair) - 1) / hb;
  const int ne_b = (int)(e1 - e0 + 1);
  for (int i = threadIdx.x; i < ne_b * kTlCols; i += kCT) {
    const int64_t e = e0 + i / kTlCols;
    const int col = i % kTlCols;
    const int64_t c0 = ck.ap_ptr[e];
    if (col < (int)(ck.ap_ptr[e + 1] - c0) * dim)
      zs[i] = (double)zc[(int64_t)ck.ap_cls[c0 + col / dim] * dim + col % dim];
  }
  __syncthreads();
  const int64_t q = q0 + threadIdx.x;
  if (q >= npair) return;
  const int64_t e = q / hb;
  const int r = 2 * (int)(q % hb);
  const int64_t c0 = ck.ap_ptr[e];
  const int ncol = (int)(ck.ap_ptr[e + 1] - c0) * dim;
  const V2 *ap = reinterpret_cast<const V2 *>(AP + c0 * dim * bu + r);
  double a0 = 0.0, a1 = 0.0;
  if (ncol <= kTlCols) {
    const double *z = zs + (e - e0) * kTlCols;
    for (int col = 0; col < ncol; ++col) {
      const V2 v = ap[(int64_t)col * hb];
      a0 += (double)v.x * z[col];
      a1 += (double)v.y * z[col];
    }
  } else {
    for (int col = 0; col < ncol; ++col) {
      const V2 v = ap[(int64_t)col * hb];
      const double zv = (double)zc[(int64_t)ck.ap_cls[c0 + col / dim] * dim + col % dim];
      a0 += (double)v.x * zv;
      a1 += (double)v.y * zv;
    }
  }
  double b0 = 0.0, b1 = 0.0;
  for (int64_t s = kp.m.sp_ptr[e]; s < kp.m.sp_ptr[e + 1]; ++s) {
    const double zv = (double)zp[kp.m.sp_pnode[s]];
    b0 += (double)Bs[s * bu + r] * zv;
    b1 += (double)Bs[s * bu + r + 1] * zv;
  }
  const int64_t t = e * bu + r;
  apz[t] = (T)a0;
  apz[t + 1] = (T)a1;
  t_out[t] = (T)((double)vu[t] - b0 - a0);
  t_out[t + 1] = (T)((double)vu[t + 1] - b1 - a1);
}

// y_p = S x_p with the dense pressure block of each instance (one wave per row)
template <typename T>
__global__ __launch_bounds__(64) void k_pgemv(KParams kp, const T *__restrict__ S, const T *__restrict__ x,
                                              T *__restrict__ y) {
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const int b = kp.pinst[i];
  const int64_t p0 = kp.poff[b], nb = kp.poff[b + 1] - p0;
  const T *row = S + kp.doff[b] + (i - p0) * nb;
  double acc = 0.0;
  for (int64_t j = lane; j < nb; j += 64) acc += (double)row[j] * (double)x[p0 + j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) y[i] = (T)acc;
}

// z_u += P z_c: thread per displacement DOF
template <typename T>
__global__ __launch_bounds__(kCT) void k_prolong_add(KParams kp, CoarseK ck, const T *__restrict__ zc,
                                                     T *__restrict__ zu) {
  const int bu = kp.s.bu, dim = ck.dim, nv = ck.nv;
  const int64_t t = blockIdx.x * (int64_t)kCT + threadIdx.x;
  if (t >= kp.s.n_u) return;
  const int64_t e = t / bu;
  const int r = (int)(t % bu), a = r / dim, comp = r % dim;
  if (clamped(kp.m.clamp, e, r)) return;
  double pz = 0.0;
  for (int v = 0; v < nv; ++v) {
    const int32_t cl = ck.cls_of[e * nv + v];
    if (cl < 0) continue;
    for (int w = 0; w < ck.nw[v]; ++w)
      if (ck.wn[v][w] == a) pz += ck.ww[v][w] * (double)zc[(int64_t)cl * dim + comp];
  }
  zu[t] = (T)((double)zu[t] + pz);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned nblk(int64_t n, int t = kCT) { return (unsigned)std::max<int64_t>((n + t - 1) / t, 1); }

hipError_t coarse_build_ap(const KParams &kp, const CoarseK &ck, const double *A, const int32_t *elist, int64_t n,
                           double *AP, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ap_build, dim3((unsigned)n), dim3(kCT), 0, st, kp, ck, A, elist, AP);
  return hipGetLastError();
}

hipError_t coarse_build_w(const KParams &kp, const CoarseK &ck, const double *Cs, const double *inv,
                          const double *AP, double *W, hipStream_t st) {
  if (kp.s.n_strip <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_w_build, dim3((unsigned)kp.s.n_strip), dim3(kCT), 0, st, kp, ck, Cs, inv, AP, W);
  return hipGetLastError();
}

hipError_t coarse_factor(const KParams &kp, const CoarseK &ck, const CoarseHostView &hv, const double *AP,
                         double *F, double *Cp, double *Dsc, int *flag, hipStream_t st) {
  hipLaunchKernelGGL(k_cfill, dim3(nblk(ck.front_total, 256) > 16384 ? 16384 : nblk(ck.front_total, 256)),
                     dim3(256), 0, st, F, ck.front_total);
  if (ck.n_pairs)
    hipLaunchKernelGGL(k_pairs, dim3(nblk(ck.n_pairs * ck.dim * ck.dim)), dim3(kCT), 0, st, kp, ck, AP, F);
  for (int l = 0; l < hv.n_levels; ++l) {
    const int nodes = hv.level_ptr[l + 1] - hv.level_ptr[l];
    if (!nodes) continue;
    if (l > 0)
      for (int slot = 0; slot < 2; ++slot) {
        const int64_t m = hv.level_maxchild_upd[l];
        if (m <= 0) break;
        const unsigned gx = (unsigned)std::min<int64_t>((m + kCT - 1) / kCT, 4096);
        hipLaunchKernelGGL(k_extend_add, dim3(gx, nodes), dim3(kCT), 0, st, ck, l, slot, F);
      }
    const int maxk = hv.level_maxk[l], maxf = hv.level_maxf[l];
    const int nt = (maxf + kTile - 1) / kTile;
    for (int p0 = 0; p0 < maxk; p0 += kNB) {
      hipLaunchKernelGGL(k_gj_a, dim3(nt, nodes), dim3(kCT), 0, st, ck, l, p0, F, Cp, Dsc, flag);
      hipLaunchKernelGGL(k_gj_b, dim3(nt * nt, nodes), dim3(kCT), 0, st, ck, l, p0, F, Cp, Dsc, flag);
    }
  }
  return hipGetLastError();
}

hipError_t coarse_ptb(const KParams &kp, const CoarseK &ck, const double *Bs, int nrhs, double *R, hipStream_t st) {
  if (!ck.ncls || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ptb, dim3(nblk((int64_t)ck.ncls * ck.dim)), dim3(kCT), 0, st, kp, ck, Bs, nrhs, R);
  return hipGetLastError();
}

template <typename TF>
hipError_t coarse_solve_multi(const CoarseK &ck, const CoarseHostView &hv, const TF *F, const double *b,
                              int nrhs, double *upd, double *y, double *xs, hipStream_t st) {
  for (int l = 0; l < hv.n_levels; ++l) {
    const int nodes = hv.level_ptr[l + 1] - hv.level_ptr[l];
    if (!nodes) continue;
    hipLaunchKernelGGL(k_fwdm_own, dim3(nblk((int64_t)hv.level_maxk[l] * nrhs), nodes), dim3(kCT), 0, st, ck, l,
                       b, upd, nrhs, y);
    const int64_t mu = (int64_t)(hv.level_maxf_minus_k[l]) * nrhs;
    if (mu > 0)
      hipLaunchKernelGGL((k_fwdm_upd<TF>), dim3(nblk(mu), nodes), dim3(kCT), 0, st, ck, l, F, y, nrhs, upd);
  }
  for (int l = hv.n_levels - 1; l >= 0; --l) {
    const int nodes = hv.level_ptr[l + 1] - hv.level_ptr[l];
    if (!nodes) continue;
    hipLaunchKernelGGL((k_bwdm<TF>), dim3(nblk((int64_t)hv.level_maxk[l] * nrhs), nodes), dim3(kCT), 0, st, ck, l, F, y,
                       nrhs, xs);
  }
  return hipGetLastError();
}

template hipError_t coarse_solve_multi<double>(const CoarseK &, const CoarseHostView &, const double *,
                                               const double *, int, double *, double *, double *, hipStream_t);
template hipError_t coarse_solve_multi<float>(const CoarseK &, const CoarseHostView &, const float *,
                                              const double *, int, double *, double *, double *, hipStream_t);

hipError_t coarse_s_correct(const KParams &kp, const CoarseK &ck, const double *W, const double *Z, int nrhs,
                            double *S, hipStream_t st) {
  if (!kp.s.n_p) return hipSuccess;
  hipLaunchKernelGGL(k_s_correct, dim3(nblk(nrhs), (unsigned)kp.s.n_p), dim3(kCT), 0, st, kp, ck, W, Z, nrhs, S);
  return hipGetLastError();
}

template <typename T, typename TF>
hipError_t coarse_solve1(const CoarseK &ck, const CoarseHostView &hv, const TF *F, const T *b, T *upd, T *y, T *cv,
                         T *xs, hipStream_t st) {
  // rows per workgroup pass: kCT / (lanes per row of the level's longest rows)
  for (int l = 0; l < hv.n_levels; ++l) {
    const int nodes = hv.level_ptr[l + 1] - hv.level_ptr[l];
    if (!nodes) continue;
    const int rpb = kCT / row_lanes(std::max(hv.level_maxk[l], 1));
    const unsigned gx = (unsigned)std::max((hv.level_maxf_minus_k[l] + rpb - 1) / rpb, 1);
    if (hv.level_maxk[l] <= kFrontLds && gx <= kFusedMaxGroups) {
      hipLaunchKernelGGL((k_fwd_fused<T, TF>), dim3(gx, nodes), dim3(kCT), 0, st, ck, l, F, b, upd, y);
      continue;
    }
    hipLaunchKernelGGL((k_fwd_own<T>), dim3((std::max(hv.level_maxk[l], 1) + kCT - 1) / kCT, nodes), dim3(kCT), 0, st, ck, l, b,
                       upd, y, cv);
    if (hv.level_maxf_minus_k[l] > 0) {
      if (hv.level_maxk[l] > kLongRow)
        hipLaunchKernelGGL((k_fwd_rows<T, TF, true>), dim3(gx, nodes), dim3(kCT), 0, st, ck, l, F, cv, upd);
      else
        hipLaunchKernelGGL((k_fwd_rows<T, TF, false>), dim3(gx, nodes), dim3(kCT), 0, st, ck, l, F, cv, upd);
    }
  }
  for (int l = hv.n_levels - 1; l >= 0; --l) {
    const int nodes = hv.level_ptr[l + 1] - hv.level_ptr[l];
    if (!nodes) continue;
    const int rpb = kCT / row_lanes(std::max(hv.level_maxf[l], 1));
    const unsigned gx = (unsigned)((std::max(hv.level_maxk[l], 1) + rpb - 1) / rpb);
    if (hv.level_maxf[l] <= kFrontLds && gx <= kFusedMaxGroups) {
      hipLaunchKernelGGL((k_bwd_fused<T, TF>), dim3(gx, nodes), dim3(kCT), 0, st, ck, l, F, y, xs);
      continue;
    }
    hipLaunchKernelGGL((k_bwd_gather<T>), dim3((std::max(hv.level_maxf[l], 1) + kCT - 1) / kCT, nodes), dim3(kCT), 0, st, ck, l,
                       y, xs, cv);
    if (hv.level_maxf[l] > kLongRow)
      hipLaunchKernelGGL((k_bwd_rows<T, TF, true>), dim3(gx, nodes), dim3(kCT), 0, st, ck, l, F, cv, xs);
    else
      hipLaunchKernelGGL((k_bwd_rows<T, TF, false>), dim3(gx, nodes), dim3(kCT), 0, st, ck, l, F, cv, xs);
  }
  return hipGetLastError();
}
template hipError_t coarse_solve1<double, double>(const CoarseK &, const CoarseHostView &, const double *,
                                                  const double *, double *, double *, double *, double *, hipStream_t);
template hipError_t coarse_solve1<double, float>(const CoarseK &, const CoarseHostView &, const float *,
                                                 const double *, double *, double *, double *, double *, hipStream_t);
template hipError_t coarse_solve1<float, float>(const CoarseK &, const CoarseHostView &, const float *, const float *,
                                                float *, float *, float *, float *, hipStream_t);

template <typename T>
hipError_t coarse_q(const KParams &kp, const CoarseK &ck, const T *Cf, const T *W, const T *vu, const T *vp,
                    const T *zc, T *qout, T *wp, hipStream_t st) {
  if (!kp.s.n_p) return hipSuccess;
  hipLaunchKernelGGL((k_tl_q<T>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp, ck, Cf, W, vu, vp, zc, qout, wp);
  return hipGetLastError();
}
template hipError_t coarse_q<double>(const KParams &, const CoarseK &, const double *, const double *,
                                     const double *, const double *, const double *, double *, double *,
                                     hipStream_t);
template hipError_t coarse_q<float>(const KParams &, const CoarseK &, const float *, const float *, const float *,
                                    const float *, const float *, float *, float *, hipStream_t);

template <typename T>
hipError_t coarse_restrict2(const KParams &kp, const CoarseK &ck, const T *v, T *cpy, T *rc, hipStream_t st) {
  if (!ck.ncls) return hipSuccess;
  hipLaunchKernelGGL((k_restrict_copies<T>), dim3(nblk(kp.s.ne * ck.nv * ck.dim)), dim3(kCT), 0, st, kp, ck, v, cpy);
  hipLaunchKernelGGL((k_restrict_gather<T>), dim3(nblk((int64_t)ck.ncls * ck.dim)), dim3(kCT), 0, st, ck, cpy, rc);
  return hipGetLastError();
}
template hipError_t coarse_restrict2<double>(const KParams &, const CoarseK &, const double *, double *, double *,
                                             hipStream_t);
template hipError_t coarse_restrict2<float>(const KParams &, const CoarseK &, const float *, float *, float *,
                                            hipStream_t);

template <typename T>
hipError_t coarse_zc2(const KParams &kp, const CoarseK &ck, const T *Z, int nrhs, const T *zc1, const T *zp, T *zc2,
                      hipStream_t st) {
  if (!ck.ncls) return hipSuccess;
  hipLaunchKernelGGL((k_zc2<T>), dim3(nblk((int64_t)ck.ncls * ck.dim, kCT / 16)), dim3(kCT), 0, st, kp, ck, Z, nrhs,
                     zc1, zp, zc2);
  return hipGetLastError();
}
template hipError_t coarse_zc2<double>(const KParams &, const CoarseK &, const double *, int, const double *,
                                       const double *, double *, hipStream_t);
template hipError_t coarse_zc2<float>(const KParams &, const CoarseK &, const float *, int, const float *,
                                      const float *, float *, hipStream_t);

template <typename T>
hipError_t coarse_t(const KParams &kp, const CoarseK &ck, const T *AP, const T *Bs, const T *vu, const T *zp,
                    const T *zc, T *t, T *apz, hipStream_t st) {
  if (kp.s.bu % 2) return hipErrorInvalidValue;  // row pairs need an even block size
  // elements a workgroup of kCT row pairs can touch: (kCT - 1) / (bu / 2) + 2
  const size_t lds = (size_t)((kCT - 1) / (kp.s.bu / 2) + 2) * kTlCols * sizeof(double);
  hipLaunchKernelGGL((k_tl_t<T>), dim3(nblk(kp.s.n_u / 2)), dim3(kCT), lds, st, kp, ck, AP, Bs, vu, zp, zc, t, apz);
  return hipGetLastError();
}
template hipError_t coarse_t<double>(const KParams &, const CoarseK &, const double *, const double *,
                                     const double *, const double *, const double *, double *, double *,
                                     hipStream_t);
template hipError_t coarse_t<float>(const KParams &, const CoarseK &, const float *, const float *, const float *,
                                    const float *, const float *, float *, float *, hipStream_t);

template <typename T>
hipError_t coarse_prolong_add(const KParams &kp, const CoarseK &ck, const T *zc, T *zu, hipStream_t st) {
  hipLaunchKernelGGL((k_prolong_add<T>), dim3(nblk(kp.s.n_u)), dim3(kCT), 0, st, kp, ck, zc, zu);
  return hipGetLastError();
}
template hipError_t coarse_prolong_add<double>(const KParams &, const CoarseK &, const double *, double *,
                                               hipStream_t);
template hipError_t coarse_prolong_add<float>(const KParams &, const CoarseK &, const float *, float *, hipStream_t);

template <typename T>
hipError_t coarse_pgemv(const KParams &kp, const T *S, const T *x, T *y, hipStream_t st) {
  if (!kp.s.n_p) return hipSuccess;
  hipLaunchKernelGGL((k_pgemv<T>), dim3((unsigned)kp.s.n_p), dim3(64), 0, st, kp, S, x, y);
  return hipGetLastError();
}
template hipError_t coarse_pgemv<double>(const KParams &, const double *, const double *, double *, hipStream_t);
template hipError_t coarse_pgemv<float>(const KParams &, const float *, const float *, float *, hipStream_t);

}  // namespace hf
