// Associate phase, second half (arXiv 2409.01712, Algorithm 3: Solve for W)
// and the FP64 pieces of refinement and Predict (Algorithm 4: P = K_test W).
//
// Triangular solves run in FP32 on the tile factor ("forward and backward
// substitution ... in the full FP32 precision", subsection on Ridge
// Regression) for all phenotype columns at once: per tile step, the
// diagonal block is applied through its inverse and the panel below (or
// beside) is updated.  The FP64 residual r = Y - (K + lambda I) X recomputes
// every kernel entry from the exact int32 distance through the FP64 table
// exp(-gamma d).
#include "common.h"
#include "internal.h"

namespace krr {

// ---------------------------------------------------------------------------
// Out[rows] (=|-=) M * V or M^T * V for one nb x nb FP32 tile M (row-major)
// and an nb x r block V (row-major, leading dimension r).  Workgroup = 64
// output rows x 32 columns; M is staged through LDS in 64 x 64 blocks.
// mode 0: M = Mbase, V = Vbase, Out = Obase (diagonal step; tri limits q)
// mode 1: forward panel, tile i = k + 1 + blockIdx.x: M = tile (i, k), Out row block i
// mode 2: backward panel, tile j = blockIdx.x: M = tile (k, j) (transposed), Out row block j
template <bool TRANS, bool SUB>
__global__ __launch_bounds__(256) void k_tri_apply(const float *__restrict__ Mbase,
                                                   const float *__restrict__ V, float *Obase,
                                                   int mode, int k, int nb, int r, int tri) {
  __shared__ float Ms[64][65];
  __shared__ float Vs[64][33];
  const int64_t te = (int64_t)nb * nb;
  const float *M = Mbase;
  float *Out = Obase;
  if (mode == 1) {
    const int64_t i = k + 1 + blockIdx.x;
    M = Mbase + (i * (i + 1) / 2 + k) * te;
    Out = Obase + i * nb * (int64_t)r;
  } else if (mode == 2) {
    const int64_t j = blockIdx.x;
    M = Mbase + ((int64_t)k * (k + 1) / 2 + j) * te;
    Out = Obase + j * nb * (int64_t)r;
  }
  const int rb = blockIdx.y, cc = blockIdx.z;
  const int tid = threadIdx.x;
  const int orow = tid >> 2, oc = (tid & 3) * 8;
  float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int q_lo = 0, q_hi = nb;
  if (tri) {  // inverse of a lower-triangular tile
    if (!TRANS) q_hi = (rb + 1) * 64;
    else q_lo = rb * 64;
  }
  for (int q0 = q_lo; q0 < q_hi; q0 += 64) {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int x = e >> 6, y = e & 63;
      if (!TRANS)
        Ms[x][y] = M[(int64_t)(rb * 64 + x) * nb + q0 + y];  // row x of the block, col q
      else
        Ms[y][x] = M[(int64_t)(q0 + x) * nb + rb * 64 + y];  // M^T: Ms[row][q] = M[q][row]
    }
    for (int e = tid; e < 64 * 32; e += 256) {
      const int x = e >> 5, y = e & 31;
      const int col = cc * 32 + y;
      Vs[x][y] = (col < r) ? V[(int64_t)(q0 + x) * r + col] : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int q = 0; q < 64; ++q) {
      const float a = Ms[orow][q];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] += a * Vs[q][oc + e];
    }
    __syncthreads();
  }
  float *o = Out + (int64_t)(rb * 64 + orow) * r;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int col = cc * 32 + oc + e;
    if (col < r) {
      if (SUB) o[col] -= acc[e];
      else o[col] = acc[e];
    }
  }
}

// L Z = B: for k: Z_k = inv(L_kk) B_k; B_i -= L_ik Z_k (i > k).
void launch_fwd_sweep(const float *Astore, const float *Linv, const TileLayout &L, int r, float *B,
                      float *Z, hipStream_t s) {
  const int nb = L.nb, NT = L.nt, RB = nb / 64, CC = (r + 31) / 32;
  const int64_t te = (int64_t)nb * nb, vb = (int64_t)nb * r;
  for (int k = 0; k < NT; ++k) {
    hipLaunchKernelGGL((k_tri_apply<false, false>), dim3(1, RB, CC), dim3(256), 0, s,
                       Linv + k * te, B + k * vb, Z + k * vb, 0, k, nb, r, 1);
    if (NT - 1 - k > 0)
      hipLaunchKernelGGL((k_tri_apply<false, true>), dim3(NT - 1 - k, RB, CC), dim3(256), 0, s,
                         Astore, Z + k * vb, B, 1, k, nb, r, 0);
  }
}

// L^T X = Z: for k descending: X_k = inv(L_kk)^T Z_k; Z_j -= L_kj^T X_k (j < k).
void launch_bwd_sweep(const float *Astore, const float *Linv, const TileLayout &L, int r, float *Z,
                      float *X, hipStream_t s) {
  const int nb = L.nb, NT = L.nt, RB = nb / 64, CC = (r + 31) / 32;
  const int64_t te = (int64_t)nb * nb, vb = (int64_t)nb * r;
  for (int k = NT - 1; k >= 0; --k) {
    hipLaunchKernelGGL((k_tri_apply<true, false>), dim3(1, RB, CC), dim3(256), 0, s,
                       Linv + k * te, Z + k * vb, X + k * vb, 0, k, nb, r, 1);
    if (k > 0)
      hipLaunchKernelGGL((k_tri_apply<true, true>), dim3(k, RB, CC), dim3(256), 0, s, Astore,
                         X + k * vb, Z, 2, k, nb, r, 0);
  }
}

// ---------------------------------------------------------------------------
// FP64 residual R = Y - (K + lambda I) X over the packed lower tiles of int32
// distances: row block (64 rows of tile row I) x 32 columns per workgroup;
// tiles (I, J <= I) are read directly and tiles (J > I, I) transposed.
__global__ __launch_bounds__(256) void k_residual(const int32_t *__restrict__ D,
                                                  const double *__restrict__ etab,
                                                  int64_t etab_len, double lambda, int64_t n,
                                                  int nb, int NT, int r,
                                                  const double *__restrict__ X,
                                                  const double *__restrict__ Y,
                                                  double *__restrict__ R) {
  __shared__ double Ks[64][65];
  __shared__ double Xs[64][33];
  const int64_t rowblk = blockIdx.x;
  const int cc = blockIdx.y;
  const int64_t g0 = rowblk * 64;
  const int I = (int)(g0 / nb), rloc = (int)(g0 % nb);
  const int tid = threadIdx.x;
  const int orow = tid >> 2, oc = (tid & 3) * 8;
  const int64_t te = (int64_t)nb * nb;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int J = 0; J < NT; ++J) {
    const bool direct = (J <= I);
    const int32_t *T = direct ? D + ((int64_t)I * (I + 1) / 2 + J) * te
                              : D + ((int64_t)J * (J + 1) / 2 + I) * te;
    for (int q0 = 0; q0 < nb; q0 += 64) {
      for (int e = tid; e < 64 * 64; e += 256) {
        const int x = e >> 6, y = e & 63;
        if (direct)
          Ks[x][y] = etab[min((int64_t)max(T[(int64_t)(rloc + x) * nb + q0 + y], 0), etab_len - 1)];
        else
          Ks[y][x] = etab[min((int64_t)max(T[(int64_t)(q0 + x) * nb + rloc + y], 0), etab_len - 1)];
      }
      for (int e = tid; e < 64 * 32; e += 256) {
        const int x = e >> 5, y = e & 31;
        const int col = cc * 32 + y;
        Xs[x][y] = (col < r) ? X[((int64_t)J * nb + q0 + x) * r + col] : 0.0;
      }
      __syncthreads();
#pragma unroll 8
      for (int q = 0; q < 64; ++q) {
        const double a = Ks[orow][q];
#pragma unroll
        for (int e = 0; e < 8; ++e) acc[e] += a * Xs[q][oc + e];
      }
      __syncthreads();
    }
  }
  const int64_t g = g0 + orow;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int col = cc * 32 + oc + e;
    if (col < r) {
      const int64_t off = g * r + col;
      R[off] = (g < n) ? Y[off] - acc[e] - lambda * X[off] : 0.0;
    }
  }
}

void launch_residual(const int32_t *D, const double *etab, int64_t etab_len, double lambda,
                     const TileLayout &L, int r, const double *X, const double *Y, double *R,
                     hipStream_t s) {
  const unsigned rb = (unsigned)(L.np / 64), cc = (unsigned)((r + 31) / 32);
  hipLaunchKernelGGL(k_residual, dim3(rb, cc), dim3(256), 0, s, D, etab, etab_len, lambda, L.n, L.nb,
                     L.nt, r, X, Y, R);
}

// Predict: P[i, :] = sum_j exp(-gamma Dt[i, j]) X[j, :] in FP64 for a block of
// test rows (Dt row-major rows x cols, X row-major cols x r).  Output written
// column-major into P (leading dimension ldp).
__global__ __launch_bounds__(256) void k_predict_apply(const int32_t *__restrict__ Dt, int64_t rows,
                                                       int64_t cols, int64_t ldd,
                                                       const double *__restrict__ etab,
                                                       int64_t etab_len,
                                                       const double *__restrict__ X, int r,
                                                       double *__restrict__ P, int64_t ldp) {
  __shared__ double Ks[64][65];
  __shared__ double Xs[64][33];
  const int64_t g0 = (int64_t)blockIdx.x * 64;
  const int cc = blockIdx.y;
  const int tid = threadIdx.x;
  const int orow = tid >> 2, oc = (tid & 3) * 8;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t q0 = 0; q0 < cols; q0 += 64) {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int x = e >> 6, y = e & 63;
      const int64_t gi = g0 + x, gj = q0 + y;
      Ks[x][y] = (gi < rows && gj < cols)
                     ? etab[min((int64_t)max(Dt[gi * ldd + gj], 0), etab_len - 1)]
                     : 0.0;
    }
    for (int e = tid; e < 64 * 32; e += 256) {
      const int x = e >> 5, y = e & 31;
      const int col = cc * 32 + y;
      Xs[x][y] = (col < r && q0 + x < cols) ? X[(q0 + x) * r + col] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int q = 0; q < 64; ++q) {
      const double a = Ks[orow][q];
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[e] += a * Xs[q][oc + e];
    }
    __syncthreads();
  }
  const int64_t g = g0 + orow;
  if (g < rows) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int col = cc * 32 + oc + e;
      if (col < r) P[(int64_t)col * ldp + g] = acc[e];
    }
  }
}

void launch_predict_apply(const int32_t *Dt, int64_t rows, int64_t cols, int64_t ldd,
                          const double *etab, int64_t etab_len, const double *X, int r, double *P,
                          int64_t ldp, hipStream_t s) {
  const unsigned rb = (unsigned)((rows + 63) / 64), cc = (unsigned)((r + 31) / 32);
  hipLaunchKernelGGL(k_predict_apply, dim3(rb, cc), dim3(256), 0, s, Dt, rows, cols, ldd, etab,
                     etab_len, X, r, P, ldp);
}

// ---------------------------------------------------------------------------
// Layout conversions and vector helpers.
__global__ void k_colmajor_to_rows(const double *__restrict__ src, int64_t n, int64_t ld, int r,
                                   int64_t np, double *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * r) return;
  const int64_t i = e / r;
  const int c = (int)(e % r);
  dst[e] = (i < n) ? src[(int64_t)c * ld + i] : 0.0;
}

void launch_colmajor_to_rows(const double *src, int64_t n, int64_t ld, int r, int64_t np,
                             double *dst, hipStream_t s) {
  const int64_t tot = np * r;
  hipLaunchKernelGGL(k_colmajor_to_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src,
                     n, ld, r, np, dst);
}

__global__ void k_rows_to_colmajor(const double *__restrict__ src, int64_t n, int r,
                                   double *__restrict__ dst, int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * r) return;
  const int64_t i = e % n;
  const int c = (int)(e / n);
  dst[(int64_t)c * ld + i] = src[i * r + c];
}

void launch_rows_to_colmajor(const double *src, int64_t n, int r, double *dst, int64_t ld,
                             hipStream_t s) {
  const int64_t tot = n * r;
  hipLaunchKernelGGL(k_rows_to_colmajor, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, src,
                     n, r, dst, ld);
}

__global__ void k_f64_to_f32(const double *__restrict__ src, int64_t count, float *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] = (float)src[e];
}

void launch_f64_to_f32(const double *src, int64_t count, float *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, src,
                     count, dst);
}

__global__ void k_axpy_f32_to_f64(const float *__restrict__ src, int64_t count, double alpha,
                                  double *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) dst[e] += alpha * (double)src[e];
}

void launch_axpy_f32_to_f64(const float *src, int64_t count, double alpha, double *dst,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_f32_to_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     src, count, alpha, dst);
}

// Squared column norms of a row-major n x r FP64 matrix, fixed order.
__global__ __launch_bounds__(256) void k_col_norms(const double *__restrict__ A, int64_t n, int r,
                                                   double *__restrict__ out) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = A[i * r + c];
    s += v * v;
  }
  s = block_sum_256(s, sh);
  if (threadIdx.x == 0) out[c] = s;
}

void launch_col_norms(const double *A, int64_t n, int r, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_col_norms, dim3(r), dim3(256), 0, s, A, n, r, out);
}

__global__ void k_fill_f64(double *p, int64_t count, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}
__global__ void k_fill_i32(int32_t *p, int64_t count, int32_t v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}
void launch_fill_f64(double *p, int64_t count, double v, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count,
                       v);
}
__global__ void k_fill_u8(uint8_t *p, int64_t count, uint8_t v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}
void launch_fill_u8(uint8_t *p, int64_t count, uint8_t v, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count,
                       v);
}
void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count,
                       v);
}

}  // namespace krr
