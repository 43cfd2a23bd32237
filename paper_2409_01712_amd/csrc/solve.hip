// Associate phase, second half (arXiv 2409.01712, Algorithm 3: Solve for W)
// and the FP64 pieces of refinement and Predict (Algorithm 4: P = K_test W).
//
// Triangular solves run in FP32 on the tile factor (the Ridge Regression
// subsection keeps both substitutions in single precision; Algorithm 3's
// Solve) for all phenotype columns at once: per tile step, the
// diagonal block is applied through its inverse and the panel below (or
// beside) is updated; one instance takes the tiles in pairs, with a
// coupling tile standing in for the step between the two.  Refinement runs
// classical iterations or conjugate gradients preconditioned by the factor.  The FP64 residual r = Y - (K + lambda I) X recomputes
// every kernel entry from the exact int32 distance through the FP64 table
// exp(-gamma d).
#include <algorithm>

#include "common.h"
#include "internal.h"

namespace krr {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Skinny products on 16 x 16 x 4 MFMA tiles.  A wavefront owns a job of 16
// output rows and 16 columns.  Lane l supplies, for each of four consecutive
// MFMAs, the A element (row l % 16, k = 4 (l / 16) + e) and the B element
// (k = 4 (l / 16) + e, column l % 16): both operands use the same k mapping,
// so each group of four MFMAs sums k over a 16-wide block exactly once.  A
// comes straight from memory (a tile of L, or exp(-gamma d) through the FP64
// table), B from the right-hand-side block, with no LDS staging.
// Output layouts (checked on the device): the FP32 16 x 16 x 4 accumulator
// holds row 4 (l / 16) + i, column l % 16 in lane l, register i; the FP64
// one holds row 4 i + l / 16, column l % 16.

// One 16 x 16 output job per workgroup: out = M[row0 .. row0+15, klo .. khi)
// V[klo .. khi, col0 .. col0+15] for an nb x nb FP32 tile M (row-major; with
// TRANS read transposed, M(row, k) = Mt[k][row]) and an nb-row block V of r
// columns, row-major (V(k, c) = V[k r + c]) or, with CM, column-major with
// column stride ldv (V(k, c) = V[c ldv + k], four k per lane in one 16-byte
// load); klo, khi multiples of 16.  The four waves take the 16-wide k
// blocks round robin, each with all its loads in flight at once (at most
// eight blocks: nb <= 512), and the partial sums are added in wave order.
// Four consecutive k of column cc of V into b (zeros when the column is past r).
template <bool CM>
__device__ __forceinline__ void load_v4(const float *V, int r, int64_t ldv, int kk, int cc,
                                        bool cv, float sg, float (&b)[4]) {
  if (CM) {
    const float4 v = *(const float4 *)(V + (int64_t)cc * ldv + kk);
    b[0] = cv ? sg * v.x : 0.f;
    b[1] = cv ? sg * v.y : 0.f;
    b[2] = cv ? sg * v.z : 0.f;
    b[3] = cv ? sg * v.w : 0.f;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float v = V[(int64_t)(kk + e) * r + cc];
      b[e] = cv ? sg * v : 0.f;
    }
  }
}

// The 16 x 16 result of a job (rows row0 + 4 (lane / 16) + e, column col) into
// o, or subtracted from it, in V's layout; lanes 0 .. 63 of the first wave.
template <bool CM, bool SUB>
__device__ __forceinline__ void store_job(float *o, int r, int64_t ldv, int row0, int col,
                                          const v4f &acc) {
  const int lane = threadIdx.x & 63;
  if (threadIdx.x >= 64 || col >= r) return;
  const int rb = row0 + 4 * (lane >> 4);
  if (CM) {
    float4 *q = (float4 *)(o + (int64_t)col * ldv + rb);
    if (SUB) {
      float4 v = *q;
      v.x -= acc[0]; v.y -= acc[1]; v.z -= acc[2]; v.w -= acc[3];
      *q = v;
    } else {
      *q = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
  } else {
    float *q = o + (int64_t)rb * r + col;
    float old[4] = {0.f, 0.f, 0.f, 0.f};
    if (SUB) {  // the four loads in flight together, then the stores
#pragma unroll
      for (int e = 0; e < 4; ++e) old[e] = q[(int64_t)e * r];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) q[(int64_t)e * r] = SUB ? old[e] - acc[e] : acc[e];
  }
}

template <bool TRANS, bool CM>
__device__ __forceinline__ v4f job_product(const float *__restrict__ M, const float *V, int nb,
                                           int r, int64_t ldv, int row0, int col0, int klo,
                                           int khi, v4f (*red)[64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int R = row0 + li, col = col0 + li;
  const int cc = min(col, r - 1);  // in-bounds load, zeroed below when col >= r
  const bool cv = col < r;
  // branch-free: blocks past khi load k block 0 (in bounds) and take zero
  // right-hand sides, so that every load is in flight before the first wait
  float a[8][4], b[8][4];
  bool okm[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k16 = klo + 16 * (wave + 4 * u);
    const bool ok = k16 < khi;
    const int kk = (ok ? k16 : 0) + 4 * lg;
    if (!TRANS) {
      const float4 v = *(const float4 *)(M + (int64_t)R * nb + kk);
      a[u][0] = v.x; a[u][1] = v.y; a[u][2] = v.z; a[u][3] = v.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) a[u][e] = M[(int64_t)(kk + e) * nb + R];
    }
    load_v4<CM>(V, r, ldv, kk, cc, true, 1.f, b[u]);
    okm[u] = cv && ok;
  }
  // all loads issued before the first use of a loaded value
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e) b[u][e] = okm[u] ? b[u][e] : 0.f;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < 8; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][e], b[u][e], acc, 0, 0, 0);
  red[wave][lane] = acc;
  __syncthreads();
  v4f sum = red[0][lane];
#pragma unroll
  for (int q = 1; q < 4; ++q) sum += red[q][lane];
  return sum;
}

// The sum of two such products, M1 V1 + sign2 M2 V2 (k ranges [klo1, khi1)
// and [klo2, khi2), multiples of 16, each at most nb <= 512 wide): the
// 16-wide k blocks of both are dealt round robin to the four waves, at most
// sixteen per wave, all loads of a wave in flight before its MFMAs.
template <bool TRANS, bool CM>
__device__ __forceinline__ v4f job_product2(const float *__restrict__ M1, const float *V1,
                                            int klo1, int khi1, const float *__restrict__ M2,
                                            const float *V2, int klo2, int khi2, float sign2,
                                            int nb, int r, int64_t ldv, int row0, int col0,
                                            v4f (*red)[64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int R = row0 + li, col = col0 + li;
  const int cc = min(col, r - 1);
  const bool cv = col < r;
  const int n1 = (khi1 - klo1) / 16, n2 = (khi2 - klo2) / 16;
  // two phases of eight blocks: half the registers of one phase of sixteen,
  // so more workgroups stay resident; the sum order over u is unchanged
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ph = 0; ph < 2; ++ph) {
    float a[8][4], b[8][4], sgm[8];
    bool okm[8];
#pragma unroll
    for (int uu = 0; uu < 8; ++uu) {
      const int g = wave + 4 * (8 * ph + uu);
      const bool first = g < n1, ok = g < n1 + n2;
      const float *M = first ? M1 : M2;
      const float *V = first ? V1 : V2;
      // branch-free as in job_product: a block past both ranges loads k
      // block 0 and takes zero right-hand sides
      const int kk = (ok ? (first ? klo1 + 16 * g : klo2 + 16 * (g - n1)) : 0) + 4 * lg;
      const float sg = first ? 1.0f : sign2;
      if (!TRANS) {
        const float4 v = *(const float4 *)(M + (int64_t)R * nb + kk);
        a[uu][0] = v.x; a[uu][1] = v.y; a[uu][2] = v.z; a[uu][3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[uu][e] = M[(int64_t)(kk + e) * nb + R];
      }
      load_v4<CM>(V, r, ldv, kk, cc, true, 1.f, b[uu]);
      okm[uu] = cv && ok;
      sgm[uu] = sg;
    }
    // all loads issued before the first use of a loaded value
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int uu = 0; uu < 8; ++uu)
#pragma unroll
      for (int e = 0; e < 4; ++e) b[uu][e] = okm[uu] ? sgm[uu] * b[uu][e] : 0.f;
#pragma unroll
    for (int uu = 0; uu < 8; ++uu)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[uu][e], b[uu][e], acc, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
  red[wave][lane] = acc;
  __syncthreads();
  v4f sum = red[0][lane];
#pragma unroll
  for (int q = 1; q < 4; ++q) sum += red[q][lane];
  return sum;
}

// Right-hand-side blocks of the sweeps: rows of tile t start at t nb r
// (row-major) or t nb (CM: column-major, column stride ldv = np).
template <bool CM>
KRR_DEV int64_t tile_off(int64_t t, int nb, int r) {
  return CM ? t * nb : t * nb * (int64_t)r;
}

// Sweep step k, diagonal part:
//   forward  Z_k = inv(L_kk) B_k     (rows of the inverse need k <= row)
//   backward X_k = inv(L_kk)^T Z_k   (its transpose, k >= row)
template <bool FWD, bool CM>
__device__ __forceinline__ void sweep_diag_body(const float *__restrict__ Linv_k, const float *In_k,
                                                float *Out_k, int nb, int r, int64_t ldv,
                                                int bid) {
  __shared__ v4f red[4][64];
  const int CJ = (r + 15) / 16;
  const int rj = bid / CJ, cj = bid % CJ;
  const int row0 = rj * 16, col0 = cj * 16;
  const v4f acc = job_product<!FWD, CM>(Linv_k, In_k, nb, r, ldv, row0, col0, FWD ? 0 : row0,
                                        FWD ? row0 + 16 : nb, red);
  store_job<CM, false>(Out_k, r, ldv, row0, col0 + (threadIdx.x & 15), acc);
}

template <bool FWD>
__global__ __launch_bounds__(256) void k_sweep_diag(const float *__restrict__ Linv_k,
                                                    const float *In_k, float *Out_k, int nb,
                                                    int r, int64_t ldv) {
  sweep_diag_body<FWD, true>(Linv_k, In_k, Out_k, nb, r, ldv, blockIdx.x);
}

// Sweep step k, update part (one job per workgroup):
//   forward  B_i -= L_ik Z_k,   i > k
//   backward Z_j -= L_kj^T X_k, j < k
template <bool FWD, bool CM>
__device__ __forceinline__ void sweep_panel_body(const float *__restrict__ Lst, const float *V_k,
                                                 float *In, int k, int nb, int r, int64_t ldv,
                                                 int64_t bid) {
  __shared__ v4f red[4][64];
  const int CJ = (r + 15) / 16, per = (nb / 16) * CJ;
  const int64_t t = bid / per;
  const int rem = (int)(bid % per), rj = rem / CJ, cj = rem % CJ;
  const int64_t i = FWD ? k + 1 + t : t;
  const int64_t te = (int64_t)nb * nb;
  const float *M = Lst + (FWD ? i * (i + 1) / 2 + k : (int64_t)k * (k + 1) / 2 + i) * te;
  const int row0 = rj * 16, col0 = cj * 16;
  const v4f acc = job_product<!FWD, CM>(M, V_k, nb, r, ldv, row0, col0, 0, nb, red);
  store_job<CM, true>(In + tile_off<CM>(i, nb, r), r, ldv, row0, col0 + (threadIdx.x & 15), acc);
}

template <bool FWD>
__global__ __launch_bounds__(256) void k_sweep_panel(const float *__restrict__ Lst,
                                                     const float *V_k, float *In, int k, int nb,
                                                     int r, int64_t ldv) {
  sweep_panel_body<FWD, true>(Lst, V_k, In, k, nb, r, ldv, blockIdx.x);
}

// Paired sweep steps over the tiles (k, k+1) = (2p, 2p+1), with the coupling
// tile C_p = inv(L_k+1,k+1) L_k+1,k inv(L_kk) standing in for the step between
// them, so that one launch covers both diagonal tiles and one the panels of both:
//   forward  Z_k = inv(L_kk) B_k,  Z_k+1 = inv(L_k+1,k+1) B_k+1 - C_p B_k,
//            B_i -= L_ik Z_k + L_i,k+1 Z_k+1,  i > k+1;
//   backward X_k+1 = inv(L_k+1,k+1)^T Z_k+1,  X_k = inv(L_kk)^T Z_k - C_p^T Z_k+1,
//            Z_j -= L_kj^T X_k + L_k+1,j^T X_k+1,  j < k.
// Right-hand sides column-major (column stride ldv).  Diagonal launch:
// 2 x per workgroups, the first per for tile k's rows.
template <bool FWD>
__global__ __launch_bounds__(256) void k_sweep_diag2(const float *__restrict__ Linv,
                                                     const float *__restrict__ Cp, const float *In,
                                                     float *Out, int k, int nb, int r,
                                                     int64_t ldv) {
  __shared__ v4f red[4][64];
  const int CJ = (r + 15) / 16, per = (nb / 16) * CJ;
  const int half = blockIdx.x / per, rem = blockIdx.x % per;
  const int rj = rem / CJ, cj = rem % CJ;
  const int row0 = rj * 16, col0 = cj * 16;
  const int64_t te = (int64_t)nb * nb;
  const float *Li0 = Linv + (int64_t)k * te, *Li1 = Linv + (int64_t)(k + 1) * te;
  const float *In0 = In + tile_off<true>(k, nb, r), *In1 = In + tile_off<true>(k + 1, nb, r);
  v4f acc;
  if (FWD) {
    if (half == 0)
      acc = job_product2<false, true>(Li0, In0, 0, row0 + 16, Cp, In0, 0, 0, 0.f, nb, r, ldv,
                                      row0, col0, red);
    else
      acc = job_product2<false, true>(Li1, In1, 0, row0 + 16, Cp, In0, 0, nb, -1.f, nb, r, ldv,
                                      row0, col0, red);
  } else {
    if (half == 1)
      acc = job_product2<true, true>(Li1, In1, row0, nb, Cp, In1, 0, 0, 0.f, nb, r, ldv, row0,
                                     col0, red);
    else
      acc = job_product2<true, true>(Li0, In0, row0, nb, Cp, In1, 0, nb, -1.f, nb, r, ldv, row0,
                                     col0, red);
  }
  store_job<true, false>(Out + tile_off<true>(k + half, nb, r), r, ldv, row0,
                         col0 + (threadIdx.x & 15), acc);
}

// x[t] for t in 0..3 through selects (a dynamic index into a local array can
// go through memory)
template <typename T, int N>
__device__ __forceinline__ T pick4(const T (&x)[N], int t) {
  return t == 0 ? x[0] : t == 1 ? x[1] : t == 2 ? x[2] : x[3];
}

// The sum of up to four products, sum_t sg[t] M_t V_t (k ranges [klo[t],
// khi[t]), multiples of 16, at most 256 values of k each): the 16-wide k
// blocks of all terms, in term order, dealt round robin to the four waves
// (at most sixteen a wave, in two phases of eight), the partial sums added
// in wave order.
template <bool TRANS>
__device__ __forceinline__ v4f job_product4(const float *const (&M)[4], const float *const (&Vp)[4],
                                            const int (&klo)[4], const int (&khi)[4],
                                            const float (&sg)[4], int nterm, int nb, int r,
                                            int64_t ldv, int row0, int col0, v4f (*red)[64]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int R = row0 + li, col = col0 + li;
  const int cc = min(col, r - 1);
  const bool cv = col < r;
  int pre[5];
  pre[0] = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) pre[t + 1] = pre[t] + (t < nterm ? (khi[t] - klo[t]) / 16 : 0);
  const int total = pre[4];
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ph = 0; ph < 2; ++ph) {
    float a[8][4], b[8][4], sgm[8];
    bool okm[8];
#pragma unroll
    for (int uu = 0; uu < 8; ++uu) {
      const int g = wave + 4 * (8 * ph + uu);
      // branch-free, the term picked by selects (no indexed local arrays): a
      // block past the last term loads k block 0 of term 0 and takes zero
      // right-hand sides, so that all loads are in flight before one wait
      const bool ok = g < total;
      const int gg = ok ? g : 0;
      const int t = (gg >= pre[1]) + (gg >= pre[2]) + (gg >= pre[3]);
      const int kk = (ok ? pick4(klo, t) + 16 * (gg - pick4(pre, t)) : 0) + 4 * lg;
      const float *Mt = pick4(M, t);
      if (!TRANS) {
        const float4 v = *(const float4 *)(Mt + (int64_t)R * nb + kk);
        a[uu][0] = v.x; a[uu][1] = v.y; a[uu][2] = v.z; a[uu][3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) a[uu][e] = Mt[(int64_t)(kk + e) * nb + R];
      }
      load_v4<true>(pick4(Vp, t), r, ldv, kk, cc, true, 1.f, b[uu]);
      okm[uu] = cv && ok;
      sgm[uu] = pick4(sg, t);
    }
    // all loads issued before the first use of a loaded value
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int uu = 0; uu < 8; ++uu)
#pragma unroll
      for (int e = 0; e < 4; ++e) b[uu][e] = okm[uu] ? sgm[uu] * b[uu][e] : 0.f;
#pragma unroll
    for (int uu = 0; uu < 8; ++uu)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[uu][e], b[uu][e], acc, 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
  red[wave][lane] = acc;
  __syncthreads();
  v4f sum = red[0][lane];
#pragma unroll
  for (int q = 1; q < 4; ++q) sum += red[q][lane];
  return sum;
}

// Quad sweep steps over the tiles k .. k+3 (k = 4q), with the block inverse
// [inv(P0) 0; -Q inv(P1)] of the quad (pairs P0, P1 with couplings C0, C1,
// inv(P) = [inv(L_a) 0; -C inv(L_b)]; Q from launch_quad_coupling):
//   forward  Z0 = iL0 B0,  Z1 = iL1 B1 - C0 B0,  Z2 = iL2 B2 - Q00 B0 - Q01 B1,
//            Z3 = iL3 B3 - C1 B2 - Q10 B0 - Q11 B1;
//   backward X3 = iL3' Z3,  X2 = iL2' Z2 - C1' Z3,  X1 = iL1' Z1 - Q01' Z2 - Q11' Z3,
//            X0 = iL0' Z0 - C0' Z1 - Q00' Z2 - Q10' Z3
// (iLj = inv(L_k+j,k+j), ' the transpose).  One launch for the four tiles:
// 4 x per workgroups, the j-th per for tile k+j's rows.  nb <= 256.
template <bool FWD>
__global__ __launch_bounds__(256) void k_sweep_diag4(const float *__restrict__ Linv,
                                                     const float *__restrict__ Cp,
                                                     const float *__restrict__ Qc, const float *In,
                                                     float *Out, int k, int nb, int r,
                                                     int64_t ldv) {
  __shared__ v4f red[4][64];
  const int CJ = (r + 15) / 16, per = (nb / 16) * CJ;
  const int j = blockIdx.x / per, rem = blockIdx.x % per;
  const int rj = rem / CJ, cj = rem % CJ;
  const int row0 = rj * 16, col0 = cj * 16;
  const int64_t te = (int64_t)nb * nb, qd = k / 4;
  const float *iL = Linv + (int64_t)(k + j) * te;
  const float *C0 = Cp + (2 * qd) * te, *C1 = Cp + (2 * qd + 1) * te;
  const float *Q = Qc + 4 * qd * te;  // Q00, Q01, Q10, Q11
  const float *V[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) V[q] = In + tile_off<true>(k + q, nb, r);
  // the terms of tile k+j: its own inverse first (its triangle), then the
  // couplings; every slot set by selects on j (no indexed stores), slots past
  // nterm empty
  const int nterm = FWD ? j + 1 : 4 - j;
  const float *M[4] = {
      iL,
      FWD ? (j == 1 ? C0 : j == 2 ? Q : C1) : (j == 2 ? C1 : j == 1 ? Q + te : C0),
      FWD ? (j == 2 ? Q + te : Q + 2 * te) : (j == 1 ? Q + 3 * te : Q),
      FWD ? Q + 3 * te : Q + 2 * te};
  const float *Vt[4] = {
      V[j], FWD ? (j == 1 ? V[0] : j == 2 ? V[0] : V[2]) : (j == 2 ? V[3] : j == 1 ? V[2] : V[1]),
      FWD ? (j == 2 ? V[1] : V[0]) : (j == 1 ? V[3] : V[2]), FWD ? V[1] : V[3]};
  const int klo[4] = {FWD ? 0 : row0, 0, 0, 0};
  const int khi[4] = {FWD ? row0 + 16 : nb, nterm > 1 ? nb : 0, nterm > 2 ? nb : 0,
                      nterm > 3 ? nb : 0};
  const float sg[4] = {1.f, -1.f, -1.f, -1.f};
  const v4f acc = job_product4<!FWD>(M, Vt, klo, khi, sg, nterm, nb, r, ldv, row0, col0, red);
  store_job<true, false>(Out + tile_off<true>(k + j, nb, r), r, ldv, row0,
                         col0 + (threadIdx.x & 15), acc);
}

// Panel launch of a pair: one job per workgroup, tile t of the panel rows
// (forward i = k+2+t; backward j = t < k).
template <bool FWD>
__global__ __launch_bounds__(256) void k_sweep_panel2(const float *__restrict__ Lst,
                                                      const float *V, float *In, int k, int nb,
                                                      int r, int64_t ldv) {
  __shared__ v4f red[4][64];
  const int CJ = (r + 15) / 16, per = (nb / 16) * CJ;
  const int64_t t = blockIdx.x / per;
  const int rem = (int)(blockIdx.x % per), rj = rem / CJ, cj = rem % CJ;
  const int64_t te = (int64_t)nb * nb;
  const int64_t i = FWD ? k + 2 + t : t;
  const float *M1 = Lst + (FWD ? tri_index(i, k) : tri_index(k, i)) * te;
  const float *M2 = Lst + (FWD ? tri_index(i, k + 1) : tri_index(k + 1, i)) * te;
  const int row0 = rj * 16, col0 = cj * 16;
  const v4f acc = job_product2<!FWD, true>(M1, V + tile_off<true>(k, nb, r), 0, nb, M2,
                                           V + tile_off<true>(k + 1, nb, r), 0, nb, 1.f, nb, r,
                                           ldv, row0, col0, red);
  store_job<true, true>(In + tile_off<true>(i, nb, r), r, ldv, row0, col0 + (threadIdx.x & 15),
                        acc);
}

// Panel launch of a pair, wide form, built for latency.  Every wave first
// issues all of its loads: the output block's current values, its share of
// the pair's 2 nb right-hand-side rows of the workgroup's 16-column block
// (1 KiB chunks straight into LDS, column stride 2 nb + 4 floats so that the
// sixteen columns an LDS read touches fall on distinct banks), and its 32 k
// blocks of L (128 floats a lane); one counter wait for the first two and
// one barrier, then each wave sums its k blocks in k order as they land.  At
// nb = 256 a wave owns a whole 16-row job (16 W rows for W waves); at
// nb = 512 two waves split a job's k range in halves, added in half order
// through LDS (8 W rows).  Columns past r read column r - 1 (their results
// are not stored).  The 16-row form needs one round trip per phase of loads
// and a reduction across all four waves.
// P tiles a step (2: a pair; 4: a quad, nb = 256): the same with P nb
// values of k, split over P nb / 512 waves a job.  t0: the launch covers
// the panel's row tiles from t0 on (forward: tile k + P + t0 first;
// backward: tile t0 first), so that a panel can be split over launches.
template <bool FWD, int NB, int W, int P = 2>
__global__ __launch_bounds__(64 * W) void k_sweep_panel2w(const float *__restrict__ Lst,
                                                          const float *V, float *In, int k, int r,
                                                          int64_t ldv, int t0) {
  typedef __attribute__((address_space(3))) void lds_void;
  constexpr int S = P * NB / 512, ROWS = 16 * W / S, RB = NB / ROWS, VST = P * NB + 4;
  constexpr int CPC = P * NB / 256, VCH = 16 * CPC / W;  // 1 KiB chunks a column; a wave
  static_assert(VCH * W == 16 * CPC && RB * ROWS == NB && S <= 2 && W % S == 0, "shape");
  extern __shared__ __attribute__((aligned(16))) float vs[];
  __shared__ v4f red[W / 2][64];
  const int CJ = (r + 15) / 16;
  const int64_t t = blockIdx.x / (RB * CJ);
  const int rem = (int)(blockIdx.x % (RB * CJ)), rj = rem / CJ, cj = rem % CJ;
  const int64_t i = FWD ? k + P + t0 + t : t0 + t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int job = wave / S, part = wave % S;
  const int row0 = rj * ROWS + job * 16, R = row0 + li;
  const int col = 16 * cj + li;
  const bool owner = part == 0 && col < r;
  float4 *q = (float4 *)(In + tile_off<true>(i, NB, r) + (int64_t)min(col, r - 1) * ldv + row0 +
                         4 * lg);
  const float4 old = *q;  // this workgroup's alone in the launch
  const float *Vk = V + tile_off<true>(k, NB, r);
#pragma unroll
  for (int u = 0; u < VCH; ++u) {
    const int h = wave + W * u, c = h / CPC, hp = h % CPC;
    const int cc = min(16 * cj + c, r - 1);
    __builtin_amdgcn_global_load_lds((const void *)(Vk + (int64_t)cc * ldv + 256 * hp + 4 * lane),
                                     (lds_void *)(vs + c * VST + 256 * hp), 16, 0, 0);
  }
  asm volatile("" ::: "memory");
  const int64_t te = (int64_t)NB * NB;
  constexpr int KBT = NB / 16;  // k blocks per tile
  // A elements of k block kb = 32 part + u (tile k + kb / KBT of the step):
  // lane (li, lg) holds M(R, 16 (kb % KBT) + 4 lg + e) of that tile, read
  // along k (forward) or down a column of the stored tile (backward,
  // transposed)
  float a[32][4];
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    const int kb = 32 * part + u, tq = kb / KBT;
    const float *M = Lst + (FWD ? tri_index(i, k + tq) : tri_index(k + tq, i)) * te;
    const int kk = 16 * (kb % KBT) + 4 * lg;
    if (FWD) {
      const float4 v = *(const float4 *)(M + (int64_t)R * NB + kk);
      a[u][0] = v.x; a[u][1] = v.y; a[u][2] = v.z; a[u][3] = v.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) a[u][e] = M[(int64_t)(kk + e) * NB + R];
    }
  }
  // the loads of L are the last 32 (forward) or 128 (backward, one float a
  // load) vector-memory operations of the wave: everything before them is done
  vm_wait<FWD ? 32 : 63>();
  bar_nofence();
  const float *vl = vs + li * VST + 4 * lg + 16 * 32 * part;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int u = 0; u < 32; ++u) {
    const float4 b = *(const float4 *)(vl + 16 * u);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][0], b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][1], b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][2], b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][3], b.w, acc, 0, 0, 0);
  }
  if (S == 2) {  // the second half's sum added to the first's
    if (part == 1) red[job][lane] = acc;
    __syncthreads();
    if (part == 0) acc += red[job][lane];
  }
  if (owner) {
    float4 v = old;
    v.x -= acc[0]; v.y -= acc[1]; v.z -= acc[2]; v.w -= acc[3];
    *q = v;
  }
}

// Panel launches of the paired sweeps: k_sweep_panel2w with 4 waves a
// workgroup, KRR_SWEEP_WIDE=8 with 8 (measured slower: a workgroup's latency
// grows with its waves a SIMD), KRR_SWEEP_WIDE=0 the 16-row form (read per
// launch).
static int sweep_wide() {
  const char *e = getenv("KRR_SWEEP_WIDE");
  if (!e) return 4;
  const int w = atoi(e);
  return w == 0 ? 0 : (w == 8 ? 8 : 4);
}

template <bool FWD, int NB, int W, int P = 2>
static void launch_panel2w(const float *Astore, const float *V, float *In, int k, int ntiles,
                           int r, int64_t ldv, hipStream_t s, int t0 = 0) {
  const size_t lds = (size_t)16 * (P * NB + 4) * sizeof(float);  // 65.8 KB at P nb = 1024
  solve_kernel_attrs();
  const int64_t blocks = (int64_t)ntiles * (NB * (P * NB / 512) / (16 * W)) * ((r + 15) / 16);
  hipLaunchKernelGGL((k_sweep_panel2w<FWD, NB, W, P>), dim3((unsigned)blocks), dim3(64 * W), lds,
                     s, Astore, V, In, k, r, ldv, t0);
}

template <bool FWD>
static void launch_panel2(const float *Astore, const float *V, float *In, int k, int ntiles,
                          int nb, int r, int64_t ldv, hipStream_t s) {
  const int w = sweep_wide();
  if (w == 4 && nb == 256) {
    launch_panel2w<FWD, 256, 4>(Astore, V, In, k, ntiles, r, ldv, s);
  } else if (w == 4 && nb == 512) {
    launch_panel2w<FWD, 512, 4>(Astore, V, In, k, ntiles, r, ldv, s);
  } else if (w && nb == 256) {
    launch_panel2w<FWD, 256, 8>(Astore, V, In, k, ntiles, r, ldv, s);
  } else if (w && nb == 512) {
    launch_panel2w<FWD, 512, 8>(Astore, V, In, k, ntiles, r, ldv, s);
  } else {
    hipLaunchKernelGGL(k_sweep_panel2<FWD>,
                       dim3((unsigned)((int64_t)ntiles * (nb / 16) * ((r + 15) / 16))), dim3(256),
                       0, s, Astore, V, In, k, nb, r, ldv);
  }
}

// The same steps for a batch of instances in lockstep (blockIdx.y = instance):
// step k of instance j runs when k < its tile count; forward B -> Z, backward
// Z -> X.  Workgroups without work return before any barrier.
template <bool FWD>
__global__ __launch_bounds__(256) void k_sweep_diag_b(const SolveJob *__restrict__ jobs, int k,
                                                      int nb, int r) {
  const SolveJob &j = jobs[blockIdx.y];
  if (k >= j.nt) return;
  const int64_t te = (int64_t)nb * nb, vb = (int64_t)nb * r;
  sweep_diag_body<FWD, false>(j.Linv + k * te, (FWD ? j.B : j.Z) + k * vb,
                              (FWD ? j.Z : j.X) + k * vb, nb, r, 0, blockIdx.x);
}

template <bool FWD>
__global__ __launch_bounds__(256) void k_sweep_panel_b(const SolveJob *__restrict__ jobs, int k,
                                                       int nb, int r) {
  const SolveJob &j = jobs[blockIdx.y];
  const int per = (nb / 16) * ((r + 15) / 16);
  const int t = (int)(blockIdx.x / per);
  if (k >= j.nt || (FWD ? k + 1 + t >= j.nt : t >= k)) return;
  const int64_t vb = (int64_t)nb * r;
  sweep_panel_body<FWD, false>(j.Lst, (FWD ? j.Z : j.X) + k * vb, FWD ? j.B : j.Z, k, nb, r, 0,
                               blockIdx.x);
}

void launch_sweeps_batched(const SolveJob *jobs, int njobs, int ntmax, int nb, int r,
                           hipStream_t s) {
  const int per = (nb / 16) * ((r + 15) / 16);
  for (int k = 0; k < ntmax; ++k) {
    hipLaunchKernelGGL(k_sweep_diag_b<true>, dim3(per, njobs), dim3(256), 0, s, jobs, k, nb, r);
    if (ntmax - 1 - k > 0)
      hipLaunchKernelGGL(k_sweep_panel_b<true>, dim3((unsigned)((ntmax - 1 - k) * per), njobs),
                         dim3(256), 0, s, jobs, k, nb, r);
  }
  for (int k = ntmax - 1; k >= 0; --k) {
    hipLaunchKernelGGL(k_sweep_diag_b<false>, dim3(per, njobs), dim3(256), 0, s, jobs, k, nb, r);
    if (k > 0)
      hipLaunchKernelGGL(k_sweep_panel_b<false>, dim3((unsigned)(k * per), njobs), dim3(256), 0, s,
                         jobs, k, nb, r);
  }
}

// L Z = B (B is overwritten), right-hand sides column-major np x r (column
// stride np).  With the coupling tiles C (nt / 2 of them, or null) the tiles
// go in pairs (0, 1), (2, 3), ..., the last one alone when nt is odd.
bool sweep_quads_supported(int nb) { return nb == 256 && sweep_wide() == 4; }

// The ordering of a split sweep: fork() lets the second stream start after
// what s holds so far (the quad's diagonal step); join_later() marks the
// launch just put on the second stream and makes s wait for the one before
// it (the two update the same tiles); join() makes s wait for the last one.
// Each record takes an event of its own.
struct SplitChain {
  const SweepSplit *sp;
  hipStream_t s;
  int used = 0;
  hipEvent_t pend = nullptr;
  SplitChain(const SweepSplit *sp_, hipStream_t s_) : sp(sp_), s(s_) {}
  bool on() const { return sp && used + 2 <= sp->nev; }
  void fork() {
    hipEvent_t e = sp->ev[used++];
    (void)hipEventRecord(e, s);
    (void)hipStreamWaitEvent(sp->s2, e, 0);
  }
  void join_later() {
    hipEvent_t e = sp->ev[used++];
    (void)hipEventRecord(e, sp->s2);
    if (pend) (void)hipStreamWaitEvent(s, pend, 0);
    pend = e;
  }
  void join() {
    if (pend) (void)hipStreamWaitEvent(s, pend, 0);
    pend = nullptr;
  }
};

void launch_fwd_sweep(const float *Astore, const float *Linv, const float *C, const float *Q,
                      const TileLayout &L, int r, float *B, float *Z, hipStream_t s,
                      const SweepSplit *sp) {
  const int nb = L.nb, NT = L.nt, CJ = (r + 15) / 16, per = (nb / 16) * CJ;
  const int64_t te = (int64_t)nb * nb, ldv = L.np;
  const bool quads = C && Q && sweep_quads_supported(nb);
  SplitChain ch(sp, s);
  for (int k = 0; k < NT;) {
    if (quads && k % 4 == 0 && k + 3 < NT) {
      hipLaunchKernelGGL(k_sweep_diag4<true>, dim3(4 * per), dim3(256), 0, s, Linv, C, Q, B, Z,
                         k, nb, r, ldv);
      const int rest = NT - 4 - k;
      if (rest > 4 && ch.on()) {
        // tiles k+8.. on the second stream once Z of this quad is out; the
        // next quad's tiles here, after the previous step's second part (both
        // update those tiles)
        ch.fork();
        launch_panel2w<true, 256, 4, 4>(Astore, Z, B, k, rest - 4, r, ldv, sp->s2, 4);
        ch.join_later();
        launch_panel2w<true, 256, 4, 4>(Astore, Z, B, k, 4, r, ldv, s, 0);
      } else if (rest > 0) {
        ch.join();
        launch_panel2w<true, 256, 4, 4>(Astore, Z, B, k, rest, r, ldv, s);
      }
      k += 4;
      continue;
    }
    ch.join();
    if (C && k + 1 < NT) {
      hipLaunchKernelGGL(k_sweep_diag2<true>, dim3(2 * per), dim3(256), 0, s, Linv,
                         C + (int64_t)(k / 2) * te, B, Z, k, nb, r, ldv);
      if (NT - 2 - k > 0) launch_panel2<true>(Astore, Z, B, k, NT - 2 - k, nb, r, ldv, s);
      k += 2;
      continue;
    }
    hipLaunchKernelGGL(k_sweep_diag<true>, dim3(per), dim3(256), 0, s, Linv + k * te,
                       B + (int64_t)k * nb, Z + (int64_t)k * nb, nb, r, ldv);
    if (NT - 1 - k > 0)
      hipLaunchKernelGGL(k_sweep_panel<true>, dim3((unsigned)((NT - 1 - k) * per)), dim3(256), 0,
                         s, Astore, Z + (int64_t)k * nb, B, k, nb, r, ldv);
    ++k;
  }
  ch.join();
}

// L^T X = Z (Z is overwritten); the pairs of the forward sweep, last first.
void launch_bwd_sweep(const float *Astore, const float *Linv, const float *C, const float *Q,
                      const TileLayout &L, int r, float *Z, float *X, hipStream_t s,
                      const SweepSplit *sp) {
  const int nb = L.nb, NT = L.nt, CJ = (r + 15) / 16, per = (nb / 16) * CJ;
  const int64_t te = (int64_t)nb * nb, ldv = L.np;
  const bool quads = C && Q && sweep_quads_supported(nb);
  SplitChain ch(sp, s);
  for (int k = NT - 1; k >= 0;) {
    if (quads && k % 4 == 3) {  // the quad (k-3 .. k) of the forward sweep
      const int k0 = k - 3;
      hipLaunchKernelGGL(k_sweep_diag4<false>, dim3(4 * per), dim3(256), 0, s, Linv, C, Q, Z, X,
                         k0, nb, r, ldv);
      if (k0 > 4 && ch.on()) {  // tiles 0 .. k0-5 on the second stream, as forward
        ch.fork();
        launch_panel2w<false, 256, 4, 4>(Astore, X, Z, k0, k0 - 4, r, ldv, sp->s2, 0);
        ch.join_later();
        launch_panel2w<false, 256, 4, 4>(Astore, X, Z, k0, 4, r, ldv, s, k0 - 4);
      } else if (k0 > 0) {
        ch.join();
        launch_panel2w<false, 256, 4, 4>(Astore, X, Z, k0, k0, r, ldv, s);
      }
      k -= 4;
      continue;
    }
    ch.join();
    if (C && k % 2 == 1) {  // the pair (k-1, k)
      const int k0 = k - 1;
      hipLaunchKernelGGL(k_sweep_diag2<false>, dim3(2 * per), dim3(256), 0, s, Linv,
                         C + (int64_t)(k0 / 2) * te, Z, X, k0, nb, r, ldv);
      if (k0 > 0) launch_panel2<false>(Astore, X, Z, k0, k0, nb, r, ldv, s);
      k -= 2;
      continue;
    }
    hipLaunchKernelGGL(k_sweep_diag<false>, dim3(per), dim3(256), 0, s, Linv + k * te,
                       Z + (int64_t)k * nb, X + (int64_t)k * nb, nb, r, ldv);
    if (k > 0)
      hipLaunchKernelGGL(k_sweep_panel<false>, dim3((unsigned)(k * per)), dim3(256), 0, s, Astore,
                         X + (int64_t)k * nb, Z, k, nb, r, ldv);
    --k;
  }
  ch.join();
}

// Row-major FP64 np x r into column-major FP32 (column stride np), and back
// as dst += alpha src: the layout changes of the sweeps' right-hand sides.
__global__ void k_rows_f64_to_cols_f32(const double *__restrict__ src, int64_t np, int r,
                                       float *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * r) return;
  const int64_t c = e / np, i = e % np;
  dst[e] = (float)src[i * r + c];
}

__global__ void k_cols_f32_axpy_rows_f64(const float *__restrict__ src, int64_t np, int r,
                                         double alpha, double *__restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * r) return;
  const int64_t c = e / np, i = e % np;
  dst[i * r + c] += alpha * (double)src[e];
}

void launch_rows_f64_to_cols_f32(const double *src, int64_t np, int r, float *dst,
                                 hipStream_t s) {
  const int64_t cnt = np * r;
  hipLaunchKernelGGL(k_rows_f64_to_cols_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s,
                     src, np, r, dst);
}

void launch_cols_f32_axpy_rows_f64(const float *src, int64_t np, int r, double alpha, double *dst,
                                   hipStream_t s) {
  const int64_t cnt = np * r;
  hipLaunchKernelGGL(k_cols_f32_axpy_rows_f64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                     s, src, np, r, alpha, dst);
}

// ---------------------------------------------------------------------------
// FP64 products with the Gaussian kernel recomputed from exact distances:
// acc[16 rows x 16 NCB cols] += sum_j exp(-gamma d(row, j)) X[j, cols].
// DMODE 0: d(row, j) = D[row * ldd + j] (row-major block)
// DMODE 1: d(row, j) = D[j * ldd + row] (transposed block)
// E (or null): factors multiplied into the kernel entries, laid out as D
// (DMODE 0 only).
template <int DMODE, int NCB, bool LIN = false>
__device__ __forceinline__ void exp_mfma_block(const int32_t *__restrict__ D, int64_t ldd, int row,
                                               int64_t j0, int64_t jn, const double *__restrict__ etab,
                                               int64_t emax, const double *__restrict__ X, int r,
                                               int64_t xrow0, int col0, int li, int lg,
                                               v4d (&acc)[NCB],
                                               const double *__restrict__ E = nullptr) {
  // j advances 64 at a time (the ranges are multiples of 64): the distance
  // loads and table lookups of four 16-wide steps are issued before their MFMAs.
  for (int64_t q = j0; q < jn; q += 64) {
    int32_t d[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t kk = q + 16 * u + 4 * lg;
      if (DMODE == 0) {
        const int4 v = *(const int4 *)(D + (int64_t)row * ldd + kk);
        d[u][0] = v.x; d[u][1] = v.y; d[u][2] = v.z; d[u][3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) d[u][e] = D[(kk + e) * ldd + row];
      }
    }
    double a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        a[u][e] = LIN ? (double)d[u][e] : etab[min((int64_t)max(d[u][e], 0), emax)];
    if (DMODE == 0 && E) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double4 f = *(const double4 *)(E + (int64_t)row * ldd + q + 16 * u + 4 * lg);
        a[u][0] *= f.x;
        a[u][1] *= f.y;
        a[u][2] *= f.z;
        a[u][3] *= f.w;
      }
    }
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      const int col = col0 + c * 16 + li;
      const int cc = min(col, r - 1);  // in-bounds load, zeroed below when col >= r
      double b[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const double v = X[(xrow0 + q - j0 + 16 * u + 4 * lg + e) * r + cc];
          b[u][e] = (col < r) ? v : 0.0;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][e], b[u][e], acc[c], 0, 0, 0);
    }
  }
}

// exp(-gamma d) without a gather per entry: with d = h W - t, h = round(d / W)
// and W a power of two, exp(-gamma d) = exp(-gamma h W) exp(gamma t), the first
// factor from a small LDS table indexed by h (the distances of a wavefront
// fall in a few neighbouring h, so the reads are broadcasts) and the second
// by its Taylor polynomial of degree RES_DEG, |gamma t| <= gamma W / 2 <=
// RES_XMAX (truncation below 2^-60 relative).  Within a few FP64 ulps of
// the correctly rounded value.
constexpr int RES_DEG = 7;
constexpr double RES_XMAX = 0.02;  // 0.02^8 / 8! < 2^-60
constexpr int RES_HI_MAX = 2048;   // entries of the LDS table

// The two tables of VM 3 from etab: ehi[h] = etab[512 h], elo[l] = etab[l]
// (EXP_LO = 512 entries), written by the whole workgroup (visible after its
// next barrier).
KRR_DEV void res_tables(const double *__restrict__ etab, int64_t dmax, double *ehi, double *elo) {
  const int nhi = (int)(dmax / EXP_LO) + 1;
  for (int q = threadIdx.x; q < EXP_LO; q += blockDim.x) elo[q] = etab[min((int64_t)q, dmax)];
  for (int q = threadIdx.x; q < nhi; q += blockDim.x) ehi[q] = etab[(int64_t)q * EXP_LO];
}

// Residual R = Y - (K + lambda I) X over the packed lower tiles of int32
// distances, in FP64 (16 x 16 x 4 MFMA).  A workgroup owns 64 rows of tile
// row I (wave w: rows 16w .. 16w+15) and 16 NCB columns, and walks all n
// columns 64 at a time: tiles (I, J <= I) are read directly, tiles (J > I, I)
// transposed.  Per 64-column step the 64 rows of X it multiplies are staged
// once in LDS for the four waves (double-buffered), and the next step's
// distances and X rows are in flight during the current step's MFMAs.
// The exponential is factored with W = 2^wshift (VM 1), or read from the FP64
// table in memory (VM 0, one gather per entry).
// VM: how a stored integer becomes the FP64 kernel value -- 0 the table
// etab[d], 1 the factored exponential above, 2 the integer itself (linear
// kernel), 3 the two-level product of LDS tables, exp(-gamma 512 h)
// exp(-gamma l) for d = 512 h + l, both factors entries of etab (the same
// values the build uses).  CONF: every kernel entry times its FP64 confounder factor Ec (the
// same packed layout as D), loaded beside the distance.
template <int NCB, int VM, bool CONF = false>
__device__ __forceinline__ void residual_body(const int32_t *__restrict__ D,
                                              const double *__restrict__ etab, int64_t etab_len,
                                              double gamma, int wshift, int64_t np, int nb, int NT,
                                              int r, const double *__restrict__ X,
                                              double *__restrict__ part, int64_t bx, int by,
                                              int bz, int nz,
                                              const double *__restrict__ Ec = nullptr) {
  constexpr int XC = 16 * NCB, XLD = XC + 2, XPT = XC / 4;  // X values per thread and step
  __shared__ double ehi[RES_HI_MAX], elo[VM == 3 ? EXP_LO : 1];
  __shared__ double xs[2][64 * XLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t dmax = etab_len - 1;
  if (VM == 1) {
    const int nhi = (int)(dmax >> wshift) + 2;
    for (int q = tid; q < nhi; q += 256) ehi[q] = exp(-gamma * (double)((int64_t)q << wshift));
  }
  if (VM == 3) res_tables(etab, dmax, ehi, elo);
  const int64_t r0 = bx * 64;  // first row of the workgroup
  const int I = (int)(r0 / nb), rloc = (int)(r0 % nb) + wave * 16;
  const int col0 = by * XC;
  const int64_t te = (int64_t)nb * nb;
  // this workgroup's share of the columns: tiles J0 .. J1-1
  const int J0 = (int)((int64_t)NT * bz / nz);
  const int J1 = (int)((int64_t)NT * (bz + 1) / nz);
  const int spt = nb / 64, st0 = J0 * spt, nsteps = J1 * spt;

  // branch-free (both orientations issue the same sixteen loads), so the
  // compiler can count them and leave the next step's loads in flight
  auto fetch_d = [&](int st, int32_t (&d)[4][4]) {
    const int J = st / spt, q = (st % spt) * 64;
    const bool dir = J <= I;
    const int64_t tb = tri_index(dir ? I : J, dir ? J : I) * te;
    const int64_t sr = dir ? nb : 1, sc = dir ? 1 : nb;  // strides of row and k
    const int32_t *b = D + tb + (int64_t)(rloc + li) * sr + (int64_t)(q + 4 * lg) * sc;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) d[u][e] = b[(int64_t)(16 * u + e) * sc];
  };
  // the confounder factors of the same entries
  auto fetch_e = [&](int st, double (&f)[4][4]) {
    const int J = st / spt, q = (st % spt) * 64;
    const bool dir = J <= I;
    const int64_t tb = tri_index(dir ? I : J, dir ? J : I) * te;
    const int64_t sr = dir ? nb : 1, sc = dir ? 1 : nb;
    const double *b = Ec + tb + (int64_t)(rloc + li) * sr + (int64_t)(q + 4 * lg) * sc;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) f[u][e] = b[(int64_t)(16 * u + e) * sc];
  };
  // element v of this thread: row (tid + 256 v) / XC, column (tid + 256 v) % XC
  auto fetch_x = [&](int st, double (&x)[XPT]) {
    const int64_t xr0 = (int64_t)(st / spt) * nb + (st % spt) * 64;
#pragma unroll
    for (int v = 0; v < XPT; ++v) {
      const int e = tid + 256 * v, t = e / XC, c = col0 + e % XC;
      const double val = X[(xr0 + t) * r + min(c, r - 1)];
      x[v] = c < r ? val : 0.0;
    }
  };
  auto store_x = [&](int buf, const double (&x)[XPT]) {
#pragma unroll
    for (int v = 0; v < XPT; ++v) {
      const int e = tid + 256 * v;
      xs[buf][(e / XC) * XLD + e % XC] = x[v];
    }
  };
  const int32_t half = VM == 1 ? (1 << wshift) >> 1 : 0;
  auto kexp = [&](int32_t d) -> double {
    if (VM == 2) return (double)d;
    const int32_t dd = (int32_t)min((int64_t)max(d, 0), dmax);
    if (VM == 0) return etab[dd];
    if (VM == 3) return exp_two_level(ehi, elo, dd);
    const int32_t h = (dd + half) >> wshift;
    const double x = gamma * (double)((h << wshift) - dd);
    double p = 1.0 / 5040.0;  // 1 / RES_DEG!
    p = fma(p, x, 1.0 / 720.0);
    p = fma(p, x, 1.0 / 120.0);
    p = fma(p, x, 1.0 / 24.0);
    p = fma(p, x, 1.0 / 6.0);
    p = fma(p, x, 0.5);
    p = fma(p, x, 1.0);
    p = fma(p, x, 1.0);
    return ehi[h] * p;
  };

  v4d acc[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) acc[c] = (v4d){0.0, 0.0, 0.0, 0.0};
  // two register sets for the distances, used alternately (no copies between
  // steps): step st computes with one while the other receives step st + 1
  int32_t da[4][4], db[4][4];
  double ea[CONF ? 4 : 1][4], eb[CONF ? 4 : 1][4];
  double xv[XPT];
  if (st0 < nsteps) {
    fetch_d(st0, da);
    if constexpr (CONF) fetch_e(st0, ea);
    fetch_x(st0, xv);
    store_x(0, xv);
  }
  __syncthreads();  // the table and the first X block
  int cur = 0;
  auto step = [&](int st, const int32_t (&dc)[4][4], int32_t (&dn)[4][4],
                  const double (&ec)[CONF ? 4 : 1][4], double (&en)[CONF ? 4 : 1][4]) {
    const bool more = st + 1 < nsteps;
    if (more) {  // X first: storing it to LDS at the end of the step waits on it alone
      fetch_x(st + 1, xv);
      fetch_d(st + 1, dn);
      if constexpr (CONF) fetch_e(st + 1, en);
    }
    double a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        a[u][e] = kexp(dc[u][e]);
        if constexpr (CONF) a[u][e] *= ec[u][e];
      }
    const double *xb = xs[cur];
#pragma unroll
    for (int c = 0; c < NCB; ++c)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              a[u][e], xb[(16 * u + 4 * lg + e) * XLD + c * 16 + li], acc[c], 0, 0, 0);
    // keep the store of the prefetched X block after this step's MFMAs (it
    // waits for those loads)
    __builtin_amdgcn_sched_barrier(0);
    if (more) store_x(cur ^ 1, xv);  // its readers (step st - 1) passed the last barrier
    // LDS reads and writes of this step done everywhere; the next step's
    // distance loads stay in flight across the barrier
    bar_nofence();
    cur ^= 1;
  };
  for (int st = st0; st < nsteps; st += 2) {
    step(st, da, db, ea, eb);
    if (st + 1 < nsteps) step(st + 1, db, da, eb, ea);
  }
  const int64_t g0 = r0 + wave * 16;
  double *P = part + (int64_t)bz * np * r;
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int col = col0 + c * 16 + li;
    if (col >= r) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) P[(g0 + 4 * i + lg) * r + col] = acc[c][i];
  }
}

// The kernel value of an integer distance (VM as in residual_body): the
// table, the factored exponential with its LDS table ehi, or the integer.
template <int VM>
KRR_DEV double res_kexp(int32_t d, const double *__restrict__ etab, int64_t dmax, double gamma,
                        int wshift, const double *ehi, const double *elo) {
  if (VM == 2) return (double)d;
  const int32_t dd = (int32_t)min((int64_t)max(d, 0), dmax);
  if (VM == 0) return etab[dd];
  if (VM == 3) return exp_two_level(ehi, elo, dd);
  const int32_t half = (1 << wshift) >> 1;
  const int32_t h = (dd + half) >> wshift;
  const double x = gamma * (double)((h << wshift) - dd);
  double p = 1.0 / 5040.0;  // 1 / RES_DEG!
  p = fma(p, x, 1.0 / 720.0);
  p = fma(p, x, 1.0 / 120.0);
  p = fma(p, x, 1.0 / 24.0);
  p = fma(p, x, 1.0 / 6.0);
  p = fma(p, x, 0.5);
  p = fma(p, x, 1.0);
  p = fma(p, x, 1.0);
  return ehi[h] * p;
}

// Residual products with every stored tile read once.  A workgroup owns the
// stored tile (I, J), I >= J (blockIdx.x in packed order), and 16 NCB columns
// of X (blockIdx.y); it walks the tile in 64 x 64 blocks (row strip a, column
// block c), turns each block's distances into FP64 kernel values once (in
// LDS), and applies them both ways with 16 x 16 x 4 FP64 MFMA:
//   R_I[strip a] += K_IJ[a, c] X_J[c]      (wave w: rows 16w ..; summed over c)
//   R_J[c]       += K_IJ[a, c]^T X_I[a]    (wave w: columns 16w .. of each c;
//                                           summed over a; I > J only)
// Each sum goes to a slot of its own, part[partner][row][col] with the other
// tile index as the partner: tile (I, J) writes slot J of the rows of I and
// slot I of the rows of J, so every (row block, partner) pair is written
// exactly once and k_residual_sum adds a row's NT slots in partner order.
// The next block's distances and X rows are loaded during the current
// block's products, and its kernel values evaluated before the barrier that
// hands the LDS block over.
template <int NCB, int VM, bool CONF>
__global__ __launch_bounds__(256) void k_residual_once(const int32_t *__restrict__ D,
                                                       const double *__restrict__ etab,
                                                       int64_t etab_len, double gamma,
                                                       int wshift, int64_t np, int nb, int r,
                                                       const double *__restrict__ X,
                                                       double *__restrict__ part,
                                                       const double *__restrict__ Ec) {
  constexpr int XC = 16 * NCB, XLD = XC + 2, XPT = XC / 4, KLD = 64 + 1;
  __shared__ double ehi[RES_HI_MAX], elo[VM == 3 ? EXP_LO : 1];
  __shared__ double ks[64 * KLD];
  __shared__ double xj[64 * XLD], xi[64 * XLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t dmax = etab_len - 1;
  if (VM == 1) {
    const int nhi = (int)(dmax >> wshift) + 2;
    for (int q = tid; q < nhi; q += 256) ehi[q] = exp(-gamma * (double)((int64_t)q << wshift));
  }
  if (VM == 3) res_tables(etab, dmax, ehi, elo);
  int I, J;
  tri_decode(blockIdx.x, I, J);
  const bool both = I != J;
  const int col0 = blockIdx.y * XC;
  const int nblk = nb / 64;
  const int64_t te = (int64_t)nb * nb;
  const int32_t *Dt = D + tri_index(I, J) * te;
  const double *Et = CONF ? Ec + tri_index(I, J) * te : nullptr;
  // this thread's 16 entries of a 64 x 64 block: row tid / 4, columns 16 (tid % 4) ..
  const int er = tid >> 2, ec = (tid & 3) * 16;
  auto fetch_d = [&](int a, int c, int32_t (&d)[16], double (&f)[CONF ? 16 : 1]) {
    const int64_t o = (int64_t)(64 * a + er) * nb + 64 * c + ec;
    const int4 *q = (const int4 *)(Dt + o);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int4 v = q[u];
      d[4 * u] = v.x; d[4 * u + 1] = v.y; d[4 * u + 2] = v.z; d[4 * u + 3] = v.w;
    }
    if constexpr (CONF) {
      const double2 *fq = (const double2 *)(Et + o);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double2 v = fq[u];
        f[2 * u] = v.x; f[2 * u + 1] = v.y;
      }
    }
  };
  // X rows row0 .. row0 + 63, columns col0 .. col0 + XC - 1 (zero past r)
  auto fetch_x = [&](int64_t row0, double (&x)[XPT]) {
#pragma unroll
    for (int v = 0; v < XPT; ++v) {
      const int e = tid + 256 * v, t = e / XC, c = col0 + e % XC;
      const double val = X[(row0 + t) * r + min(c, r - 1)];
      x[v] = c < r ? val : 0.0;
    }
  };
  auto store_x = [&](double *xs, const double (&x)[XPT]) {
#pragma unroll
    for (int v = 0; v < XPT; ++v) {
      const int e = tid + 256 * v;
      xs[(e / XC) * XLD + e % XC] = x[v];
    }
  };
  auto kvals = [&](const int32_t (&d)[16], const double (&f)[CONF ? 16 : 1], double (&kv)[16]) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      kv[q] = res_kexp<VM>(d[q], etab, dmax, gamma, wshift, ehi, elo);
      if constexpr (CONF) kv[q] *= f[q];
    }
  };
  auto store_k = [&](const double (&kv)[16]) {
#pragma unroll
    for (int q = 0; q < 16; ++q) ks[er * KLD + ec + q] = kv[q];
  };

  v4d acc_t[8][NCB];
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int b = 0; b < NCB; ++b) acc_t[c][b] = (v4d){0.0, 0.0, 0.0, 0.0};
  int32_t dn[16];
  double fn[CONF ? 16 : 1], kv[16], xn[XPT], xin[XPT];
  __syncthreads();  // the exponential table
  // block (0, 0) into LDS
  fetch_d(0, 0, dn, fn);
  fetch_x((int64_t)J * nb, xn);
  fetch_x((int64_t)I * nb, xin);
  kvals(dn, fn, kv);
  store_k(kv);
  store_x(xj, xn);
  store_x(xi, xin);
  __syncthreads();
  for (int a = 0; a < nblk; ++a) {
    v4d acc_d[NCB], acc_e[NCB];
#pragma unroll
    for (int b = 0; b < NCB; ++b) acc_d[b] = acc_e[b] = (v4d){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c >= nblk) break;
      // the next block: (a, c + 1), or the next strip's first block
      const int na = c + 1 < nblk ? a : a + 1, nc = c + 1 < nblk ? c + 1 : 0;
      const bool more = na < nblk;
      if (more) {
        fetch_x((int64_t)J * nb + 64 * nc, xn);
        if (nc == 0) fetch_x((int64_t)I * nb + 64 * na, xin);
        fetch_d(na, nc, dn, fn);
      }
      // R_I[strip a] += K[a, c] X_J[c] and R_J[c] += K[a, c]^T X_I[a], the
      // MFMAs of the two sums interleaved (independent accumulators, so each
      // chain's latency is hidden behind the other); the diagonal tile splits
      // its direct sum over two accumulators (even and odd k) instead
      if (both) {
#pragma unroll
        for (int b = 0; b < NCB; ++b)
#pragma unroll
          for (int k0 = 0; k0 < 64; k0 += 4) {
            acc_d[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                ks[(16 * wave + li) * KLD + k0 + lg], xj[(k0 + lg) * XLD + 16 * b + li],
                acc_d[b], 0, 0, 0);
            acc_t[c][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                ks[(k0 + lg) * KLD + 16 * wave + li], xi[(k0 + lg) * XLD + 16 * b + li],
                acc_t[c][b], 0, 0, 0);
          }
      } else {
#pragma unroll
        for (int b = 0; b < NCB; ++b)
#pragma unroll
          for (int k0 = 0; k0 < 64; k0 += 8) {
            acc_d[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                ks[(16 * wave + li) * KLD + k0 + lg], xj[(k0 + lg) * XLD + 16 * b + li],
                acc_d[b], 0, 0, 0);
            acc_e[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                ks[(16 * wave + li) * KLD + k0 + 4 + lg], xj[(k0 + 4 + lg) * XLD + 16 * b + li],
                acc_e[b], 0, 0, 0);
          }
      }
      if (more) kvals(dn, fn, kv);
      __syncthreads();  // every wave is done with this block's LDS
      if (more) {
        store_k(kv);
        store_x(xj, xn);
        if (nc == 0) store_x(xi, xin);
      }
      __syncthreads();
    }
    // the direct sum of strip a: slot J of rows I nb + 64 a + 16 wave ..
    if (!both) {
#pragma unroll
      for (int b = 0; b < NCB; ++b) acc_d[b] += acc_e[b];
    }
    double *P = part + (int64_t)J * np * r;
    const int64_t g0 = (int64_t)I * nb + 64 * a + 16 * wave;
#pragma unroll
    for (int b = 0; b < NCB; ++b) {
      const int col = col0 + 16 * b + li;
      if (col >= r) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) P[(g0 + 4 * i + lg) * r + col] = acc_d[b][i];
    }
  }
  if (both) {
    // the transposed sums: slot I of rows J nb + 64 c + 16 wave ..
    double *P = part + (int64_t)I * np * r;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (c >= nblk) break;
      const int64_t g0 = (int64_t)J * nb + 64 * c + 16 * wave;
#pragma unroll
      for (int b = 0; b < NCB; ++b) {
        const int col = col0 + 16 * b + li;
        if (col >= r) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) P[(g0 + 4 * i + lg) * r + col] = acc_t[c][b][i];
      }
    }
  }
}

template <int NCB, int VM, bool CONF>
__global__ __launch_bounds__(256) void k_residual(const int32_t *__restrict__ D,
                                                  const double *__restrict__ etab,
                                                  int64_t etab_len, double gamma, int wshift,
                                                  int64_t np, int nb, int NT, int r,
                                                  const double *__restrict__ X,
                                                  double *__restrict__ part,
                                                  const double *__restrict__ Ec) {
  residual_body<NCB, VM, CONF>(D, etab, etab_len, gamma, wshift, np, nb, NT, r, X, part,
                                 blockIdx.x, blockIdx.y, blockIdx.z, gridDim.z, Ec);
}

// All instances of a batch in one launch: blockIdx.x runs over the row
// blocks of every instance (the job owning it found by its first block),
// blockIdx.z over the column split, cut to the instance's own split.
template <int NCB, int VM>
__global__ __launch_bounds__(256) void k_residual_b(const SolveJob *__restrict__ jobs, int njobs,
                                                    int nb, int r) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].rb0 <= (int64_t)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const SolveJob &j = jobs[lo];
  const int nz = j.nt < 4 ? j.nt : 4;  // residual_split_batched
  if ((int)blockIdx.z >= nz) return;
  residual_body<NCB, VM>(j.D, j.etab, j.etab_len, j.gamma, j.wshift, j.np, nb, j.nt, r, j.Xd,
                           j.part, (int64_t)blockIdx.x - j.rb0, blockIdx.y, blockIdx.z, nz);
}

// R = Y - sum_z part[z] - lambda X, the partial products added in z order.
__global__ void k_residual_sum(const double *__restrict__ part, int nsplit, int64_t np, int r,
                               int64_t n, double lambda, const double *__restrict__ X,
                               const double *__restrict__ Y, double *__restrict__ R) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= np * r) return;
  double s = 0.0;
  for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * np * r + e];
  R[e] = (e / r < n) ? Y[e] - s - lambda * X[e] : 0.0;
}

// log2 of the largest W = 2^k with gamma W / 2 <= RES_XMAX whose table of
// exp(-gamma h W), h <= dmax / W + 1, fits in LDS; -1 when none does.
static int residual_wshift(double gamma, int64_t dmax) {
  int k = 0;
  while (k < 30 && gamma * (double)(1LL << (k + 1)) * 0.5 <= RES_XMAX) ++k;
  if (gamma * (double)(1LL << k) * 0.5 > RES_XMAX) return -1;
  if ((dmax >> k) + 2 > RES_HI_MAX) return -1;
  return k;
}

// Tile-column ranges of the residual's partial products: 8 for one instance
// (measured at n = 32768: 5.25 ms per step with 4, 5.03 with 8, 4.99 with 16,
// 5.64 with 2), 4 in the lockstep batch (its grid already has many instances).
int residual_split(const TileLayout &L) { return std::min(8, L.nt); }
int residual_split_batched(const TileLayout &L) { return std::min(4, L.nt); }
int residual_exp_shift(double gamma, int64_t etab_len) {
  return residual_wshift(gamma, etab_len - 1);
}

// The two-level tables (VM 3) fit in LDS, and are not switched off
// (KRR_RES_EXP=taylor keeps the factored exponential of VM 1).
static bool residual_two_level(int64_t etab_len) {
  static const bool taylor = [] {
    const char *e = getenv("KRR_RES_EXP");
    return e && e[0] == 't';
  }();
  return !taylor && (etab_len - 1) / EXP_LO + 1 <= RES_HI_MAX;
}

void launch_residual_batched(const SolveJob *jobs, int njobs, int64_t rblocks, bool fact, int nb,
                             int r, hipStream_t s) {
  const int ncb = (r + 15) / 16;
  const dim3 grid((unsigned)rblocks, ncb <= 2 ? 1u : (unsigned)((r + 63) / 64), 4);
#define KRR_RESB(NCB, VM)                                                                    \
  hipLaunchKernelGGL((k_residual_b<NCB, VM>), grid, dim3(256), 0, s, jobs, njobs, nb, r)
  if (fact) {
    if (ncb <= 1) KRR_RESB(1, 1);
    else if (ncb <= 2) KRR_RESB(2, 1);
    else KRR_RESB(4, 1);
  } else {
    if (ncb <= 1) KRR_RESB(1, 0);
    else if (ncb <= 2) KRR_RESB(2, 0);
    else KRR_RESB(4, 0);
  }
#undef KRR_RESB
}

void launch_residual_sum(const double *part, int nsplit, const TileLayout &L, int r,
                         double lambda, const double *X, const double *Y, double *R,
                         hipStream_t s) {
  const int64_t tot = L.np * r;
  hipLaunchKernelGGL(k_residual_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part,
                     nsplit, L.np, r, L.n, lambda, X, Y, R);
}

void launch_residual(const int32_t *D, const double *etab, int64_t etab_len, double gamma,
                     int vmode, const double *Ec, double lambda, const TileLayout &L, int r,
                     const double *X, const double *Y, double *R, double *part, int nsplit,
                     hipStream_t s) {
  const unsigned rb = (unsigned)(L.np / 64);
  const int ncb = (r + 15) / 16, z = std::max(1, std::min(nsplit, L.nt));
  const int ws = vmode == VAL_EXP ? residual_wshift(gamma, etab_len - 1) : -1;
  const bool two = vmode == VAL_EXP && residual_two_level(etab_len);
  const dim3 grid(rb, ncb <= 2 ? 1u : (unsigned)((r + 63) / 64), z);
#define KRR_RES(NCB, VM, CONF)                                                      \
  hipLaunchKernelGGL((k_residual<NCB, VM, CONF>), grid, dim3(256), 0, s, D, etab, etab_len, \
                     gamma, ws, L.np, L.nb, L.nt, r, X, part, Ec)
#define KRR_RES2(VM, CONF)              \
  do {                                     \
    if (ncb <= 1) KRR_RES(1, VM, CONF);  \
    else if (ncb <= 2) KRR_RES(2, VM, CONF); \
    else KRR_RES(4, VM, CONF);           \
  } while (0)
  if (vmode == VAL_LINEAR) {
    KRR_RES2(2, false);
  } else if (Ec) {
    if (two) KRR_RES2(3, true);
    else if (ws >= 0) KRR_RES2(1, true);
    else KRR_RES2(0, true);
  } else {
    if (two) KRR_RES2(3, false);
    else if (ws >= 0) KRR_RES2(1, false);
    else KRR_RES2(0, false);
  }
#undef KRR_RES2
#undef KRR_RES
  const int64_t tot = L.np * r;
  hipLaunchKernelGGL(k_residual_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part, z,
                     L.np, r, L.n, lambda, X, Y, R);
}

// Bytes of the slots of the read-once residual (NT partners per row block).
int64_t residual_once_bytes(const TileLayout &L, int r) { return (int64_t)L.nt * L.np * r * 8; }

void launch_residual_once(const int32_t *D, const double *etab, int64_t etab_len, double gamma,
                          int vmode, const double *Ec, double lambda, const TileLayout &L, int r,
                          const double *X, const double *Y, double *R, double *part,
                          hipStream_t s) {
  const int ncb = r <= 16 ? 1 : 2, xc = 16 * ncb;
  const int ws = vmode == VAL_EXP ? residual_wshift(gamma, etab_len - 1) : -1;
  const bool two = vmode == VAL_EXP && residual_two_level(etab_len);
  const dim3 grid((unsigned)L.ntiles(), (unsigned)((r + xc - 1) / xc));
#define KRR_RO(NCB, VM, CONF)                                                                 \
  hipLaunchKernelGGL((k_residual_once<NCB, VM, CONF>), grid, dim3(256), 0, s, D, etab,         \
                     etab_len, gamma, ws, L.np, L.nb, r, X, part, Ec)
#define KRR_RO2(VM, CONF)              \
  do {                                  \
    if (ncb == 1) KRR_RO(1, VM, CONF);  \
    else KRR_RO(2, VM, CONF);           \
  } while (0)
  if (vmode == VAL_LINEAR) {
    KRR_RO2(2, false);
  } else if (Ec) {
    if (two) KRR_RO2(3, true);
    else if (ws >= 0) KRR_RO2(1, true);
    else KRR_RO2(0, true);
  } else {
    if (two) KRR_RO2(3, false);
    else if (ws >= 0) KRR_RO2(1, false);
    else KRR_RO2(0, false);
  }
#undef KRR_RO2
#undef KRR_RO
  const int64_t tot = L.np * r;
  hipLaunchKernelGGL(k_residual_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, part,
                     L.nt, L.np, r, L.n, lambda, X, Y, R);
}

// Predict: P[i, :] = sum_j exp(-gamma Dt[i, j]) X[j, :] in FP64 for a block of
// test rows (Dt row-major rows x cols, cols a multiple of 16; X row-major
// cols x r).  Output written column-major into P (leading dimension ldp).
template <int NCB, bool LIN>
__global__ __launch_bounds__(256) void k_predict_apply(const int32_t *__restrict__ Dt, int64_t rows,
                                                       int64_t cols, int64_t ldd,
                                                       const double *__restrict__ etab,
                                                       int64_t etab_len,
                                                       const double *__restrict__ X, int r,
                                                       double *__restrict__ P, int64_t ldp,
                                                       const double *__restrict__ Et) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t g0 = (int64_t)blockIdx.x * 64 + wave * 16;
  const int col0 = blockIdx.y * 16 * NCB;
  v4d acc[NCB];
#pragma unroll
  for (int c = 0; c < NCB; ++c) acc[c] = (v4d){0.0, 0.0, 0.0, 0.0};
  // rows past the end read row rows-1 (valid memory); their outputs are dropped
  const int64_t arow = min(g0 + li, rows - 1);
  exp_mfma_block<0, NCB, LIN>(Dt + arow * ldd, ldd, 0, 0, cols, etab, etab_len - 1, X, r, 0, col0,
                              li, lg, acc, Et ? Et + arow * ldd : nullptr);
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    const int col = col0 + c * 16 + li;
    if (col >= r) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t g = g0 + 4 * i + lg;
      if (g < rows) P[(int64_t)col * ldp + g] = acc[c][i];
    }
  }
}

void launch_predict_apply(const int32_t *Dt, int64_t rows, int64_t cols, int64_t ldd,
                          const double *etab, int64_t etab_len, const double *X, int r, double *P,
                          int64_t ldp, const double *Et, bool linear, hipStream_t s) {
  const unsigned rb = (unsigned)((rows + 63) / 64);
  const int ncb = (r + 15) / 16;
#define KRR_PA(NCB, LIN, GY)                                                                      \
  hipLaunchKernelGGL((k_predict_apply<NCB, LIN>), dim3(rb, GY), dim3(256), 0, s, Dt, rows, cols, \
                     ldd, etab, etab_len, X, r, P, ldp, Et)
  const unsigned gy = (unsigned)((r + 63) / 64);
  if (linear) {
    if (ncb <= 1) KRR_PA(1, true, 1);
    else if (ncb <= 2) KRR_PA(2, true, 1);
    else KRR_PA(4, true, gy);
  } else {
    if (ncb <= 1) KRR_PA(1, false, 1);
    else if (ncb <= 2) KRR_PA(2, false, 1);
    else KRR_PA(4, false, gy);
  }
#undef KRR_PA
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

// Column dot products sum_i A_ic B_ic of two row-major n x r FP64 matrices
// (squared column norms when B = A), in a fixed order: COL_SPLIT slices of
// rows summed per column by one workgroup each into ws, then the slices
// added in slice order.
constexpr int COL_SPLIT = 32;

__global__ __launch_bounds__(256) void k_col_dots_part(const double *__restrict__ A,
                                                       const double *__restrict__ B, int64_t n,
                                                       int r, double *__restrict__ ws) {
  __shared__ double sh[4];
  const int c = blockIdx.x, sl = blockIdx.y;
  const int64_t i0 = n * sl / COL_SPLIT, i1 = n * (sl + 1) / COL_SPLIT;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) s += A[i * r + c] * B[i * r + c];
  s = block_sum<4>(s, sh);
  if (threadIdx.x == 0) ws[(int64_t)sl * r + c] = s;
}

__global__ void k_col_dots_sum(const double *__restrict__ ws, int r, double *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= r) return;
  double s = 0.0;
  for (int sl = 0; sl < COL_SPLIT; ++sl) s += ws[(int64_t)sl * r + c];
  out[c] = s;
}

int col_dots_workspace(int r) { return COL_SPLIT * r; }

void launch_col_dots(const double *A, const double *B, int64_t n, int r, double *out, double *ws,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_col_dots_part, dim3(r, COL_SPLIT), dim3(256), 0, s, A, B, n, r, ws);
  hipLaunchKernelGGL(k_col_dots_sum, dim3((r + 255) / 256), dim3(256), 0, s, ws, r, out);
}

void launch_col_norms(const double *A, int64_t n, int r, double *out, double *ws, hipStream_t s) {
  launch_col_dots(A, A, n, r, out, ws, s);
}

// One step of conjugate gradients on every column c of row-major n x r
// matrices, given nq = -A p (the residual kernel with a zero right-hand side):
//   alpha_c = rho_c / (p_c . A p_c),  x_c += alpha_c p_c,  r_c -= alpha_c A p_c.
// A zero curvature (only when p_c = 0) gives alpha_c = 0.
__global__ void k_pcg_step(double *__restrict__ x, double *__restrict__ res,
                           const double *__restrict__ p, const double *__restrict__ nq,
                           const double *__restrict__ rho, const double *__restrict__ pnq,
                           int64_t count, int r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int c = (int)(e % r);
  const double den = -pnq[c];
  const double alpha = den != 0.0 ? rho[c] / den : 0.0;
  x[e] += alpha * p[e];
  res[e] += alpha * nq[e];
}

void launch_pcg_step(double *x, double *res, const double *p, const double *nq, const double *rho,
                     const double *pnq, int64_t count, int r, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_step, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, x, res, p,
                     nq, rho, pnq, count, r);
}

// New search directions p_c = z_c + beta_c p_c, beta_c = rho_new_c / rho_old_c
// (0 when rho_old_c is 0); start: rho_old = nullptr gives p = z.
__global__ void k_pcg_dir(double *__restrict__ p, const double *__restrict__ z,
                          const double *__restrict__ rho_new, const double *__restrict__ rho_old,
                          int64_t count, int r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int c = (int)(e % r);
  double beta = 0.0;
  if (rho_old && rho_old[c] != 0.0) beta = rho_new[c] / rho_old[c];
  p[e] = z[e] + beta * p[e];
}

void launch_pcg_dir(double *p, const double *z, const double *rho_new, const double *rho_old,
                    int64_t count, int r, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_dir, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, z,
                     rho_new, rho_old, count, r);
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

// Dynamic-LDS limits of the wide sweep panels (65.8 KB at nb = 512, above the
// 64 KB default), set once per process before their first launch; the
// context's creation calls it, so that it never runs inside a stream capture.
void solve_kernel_attrs() {
  static bool done = false;
  if (done) return;
  done = true;
  const int l256 = 16 * (2 * 256 + 4) * (int)sizeof(float);
  const int l512 = 16 * (2 * 512 + 4) * (int)sizeof(float);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<true, 256, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l256);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<false, 256, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l256);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<true, 256, 8>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l256);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<false, 256, 8>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l256);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<true, 512, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l512);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<false, 512, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l512);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<true, 512, 8>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l512);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<false, 512, 8>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l512);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<true, 256, 4, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l512);
  (void)hipFuncSetAttribute((const void *)k_sweep_panel2w<false, 256, 4, 4>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, l512);
}

}  // namespace krr
