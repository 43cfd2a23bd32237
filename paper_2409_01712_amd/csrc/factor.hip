// Associate phase, first half: tile Cholesky of K + lambda*I with a
// per-update choice of operand precision (arXiv 2409.01712, Algorithm 3;
// "Deploying a Four-Precision Cholesky-Based Solver").
//
// Right-looking over panels k = 0 .. NT-1:
//   POTRF   L_kk = chol(A_kk) in FP64 (or FP32 on the plain path), with
//           L_kk^{-1} formed alongside;
//   TRSM    L_ik = A_ik L_kk^{-T} as an FP32 MFMA product with L_kk^{-1};
//   convert L_ik to FP16 / FP8 E4M3 copies with a per-tile power-of-two
//           scale (produced once per panel, consumed by every update);
//   update  A_ij -= L_ik L_jk^T for k < j <= i: FP32 on diagonal tiles and
//           early panels, otherwise FP16 or FP8 operands chosen per update
//           from the operand tile norms, always accumulated in FP32.
#include "common.h"
#include "internal.h"

namespace krr {

constexpr int BS = 64;  // sub-block of the diagonal-tile factorization

// ---------------------------------------------------------------------------
// Diagonal tile: blocked Cholesky and triangular inverse, 64 x 64 sub-blocks.
// W holds the nb x nb tile (row-major) in T = double or float.

template <typename T>
__global__ void k_potrf_load(const float *__restrict__ Akk, T *__restrict__ W, int nb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * nb) return;
  const int r = (int)(e / nb), c = (int)(e % nb);
  W[e] = (c <= r) ? (T)Akk[e] : (T)0;
}

// Factor sub-block (s, s) and invert it with one wavefront (64 lanes, so a
// workgroup barrier is only a wave barrier).  Lane i owns row i of the block
// during the factorization and column i of the inverse afterwards; both
// live in LDS, and every cross-lane read is a broadcast of one element.
template <typename T>
__global__ __launch_bounds__(64) void k_potrf_diag64(T *__restrict__ W, int nb, int s,
                                                     T *__restrict__ Dinv, int32_t *flag,
                                                     int64_t colbase) {
  __shared__ T L[BS][BS + 1];
  __shared__ T Li[BS][BS + 1];
  const int i = threadIdx.x;
  T *blk = W + (int64_t)(s * BS) * nb + s * BS;
  for (int e = i; e < BS * BS; e += BS) {
    const int r = e / BS, c = e % BS;
    L[r][c] = (c <= r) ? blk[(int64_t)r * nb + c] : (T)0;
  }
  __syncthreads();
  for (int j = 0; j < BS; ++j) {
    const T piv = L[j][j];
    const bool bad = !(piv > (T)0);
    const T d = bad ? (T)1 : sqrt(piv);
    __syncthreads();
    T lij = (T)0;
    if (i > j) {
      lij = L[i][j] / d;
      L[i][j] = lij;
    } else if (i == j) {
      L[j][j] = d;
      if (bad) atomicCAS(flag, 0, (int32_t)(colbase + s * BS + j + 1));
    }
    __syncthreads();
    if (i > j) {
#pragma unroll 4
      for (int c = j + 1; c <= i; ++c) L[i][c] -= lij * L[c][j];
    }
    __syncthreads();
  }
  // column c = i of inv(L) by forward substitution against e_c
  const int c = i;
  for (int k = 0; k < BS; ++k) {
    T acc0 = (k == c) ? (T)1 : (T)0, acc1 = 0, acc2 = 0, acc3 = 0;
    int p = c;
    for (; p + 3 < k; p += 4) {
      acc0 -= L[k][p] * Li[p][c];
      acc1 -= L[k][p + 1] * Li[p + 1][c];
      acc2 -= L[k][p + 2] * Li[p + 2][c];
      acc3 -= L[k][p + 3] * Li[p + 3][c];
    }
    for (; p < k; ++p) acc0 -= L[k][p] * Li[p][c];
    Li[k][c] = (k < c) ? (T)0 : ((acc0 + acc1) + (acc2 + acc3)) / L[k][k];
  }
  __syncthreads();
  for (int e = i; e < BS * BS; e += BS) {
    const int r = e / BS, cc = e % BS;
    Dinv[(int64_t)s * BS * BS + e] = Li[r][cc];
    blk[(int64_t)r * nb + cc] = (cc <= r) ? L[r][cc] : (T)0;
  }
}

// 64x64x64 product helper: each of 256 threads owns a 4 x 4 output patch.
// acc[a][b] += sum_p X[r0 + a][p] * Y(p, c0 + b), where Y(p, c) = Yt[c][p]
// if YT (Y given transposed) else Yt[p][c].
template <typename T, bool YT>
__device__ __forceinline__ void mm64(const T (*X)[BS + 1], const T (*Yt)[BS + 1], T (&acc)[4][4],
                                     int r0, int c0) {
  for (int p = 0; p < BS; ++p) {
    T xa[4], yb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) xa[a] = X[r0 + a][p];
#pragma unroll
    for (int b = 0; b < 4; ++b) yb[b] = YT ? Yt[c0 + b][p] : Yt[p][c0 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * yb[b];
  }
}

// Stage a 64 x 64 block into LDS: all 16 loads of a thread are issued before
// any LDS store, so their latencies overlap.
template <typename T>
__device__ __forceinline__ void load64(T (*dst)[BS + 1], const T *src, int64_t ld) {
  constexpr int PER = BS * BS / 256;
  T v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * 256;
    v[q] = src[(int64_t)(e / BS) * ld + e % BS];
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * 256;
    dst[e / BS][e % BS] = v[q];
  }
}

// Panel of the diagonal tile: W_as <- W_as * inv(L_ss)^T for a > s.
template <typename T>
__global__ __launch_bounds__(256) void k_potrf_trsm64(T *__restrict__ W, int nb, int s,
                                                      const T *__restrict__ Dinv) {
  __shared__ T X[BS][BS + 1];
  __shared__ T Li[BS][BS + 1];
  const int a = s + 1 + blockIdx.x;
  T *blk = W + (int64_t)(a * BS) * nb + s * BS;
  load64(X, blk, nb);
  load64(Li, Dinv + (int64_t)s * BS * BS, BS);
  __syncthreads();
  const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
  T acc[4][4] = {};
  mm64<T, true>(X, Li, acc, r0, c0);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) blk[(int64_t)(r0 + i) * nb + c0 + j] = acc[i][j];
}

// Trailing update inside the diagonal tile: W_ab -= W_as W_bs^T, s < b <= a.
template <typename T>
__global__ __launch_bounds__(256) void k_potrf_syrk64(T *__restrict__ W, int nb, int s) {
  __shared__ T Xa[BS][BS + 1];
  __shared__ T Xb[BS][BS + 1];
  int a, b;
  tri_decode(blockIdx.x, a, b);
  a += s + 1;
  b += s + 1;
  load64(Xa, W + (int64_t)(a * BS) * nb + s * BS, nb);
  load64(Xb, W + (int64_t)(b * BS) * nb + s * BS, nb);
  __syncthreads();
  const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
  T acc[4][4] = {};
  mm64<T, true>(Xa, Xb, acc, r0, c0);
  T *blk = W + (int64_t)(a * BS) * nb + b * BS;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) blk[(int64_t)(r0 + i) * nb + c0 + j] -= acc[i][j];
}

// Off-diagonal blocks of inv(L) at block distance delta = a - b:
// Winv_ab = -inv(L_aa) * sum_{c=b}^{a-1} L_ac Winv_cb, with Winv_bb = inv(L_bb).
template <typename T>
__global__ __launch_bounds__(256) void k_trtri_off64(const T *__restrict__ W, T *__restrict__ Winv,
                                                     int nb, int delta,
                                                     const T *__restrict__ Dinv) {
  __shared__ T X[BS][BS + 1];
  __shared__ T Y[BS][BS + 1];
  const int b = blockIdx.x, a = b + delta;
  const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
  T acc[4][4] = {};
  for (int c = b; c < a; ++c) {
    load64(X, W + (int64_t)(a * BS) * nb + c * BS, nb);
    if (c == b)
      load64(Y, Dinv + (int64_t)b * BS * BS, BS);
    else
      load64(Y, Winv + (int64_t)(c * BS) * nb + b * BS, nb);
    __syncthreads();
    mm64<T, false>(X, Y, acc, r0, c0);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) X[r0 + i][c0 + j] = acc[i][j];
  load64(Y, Dinv + (int64_t)a * BS * BS, BS);
  __syncthreads();
  T out[4][4] = {};
  mm64<T, false>(Y, X, out, r0, c0);
  T *blk = Winv + (int64_t)(a * BS) * nb + b * BS;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) blk[(int64_t)(r0 + i) * nb + c0 + j] = -out[i][j];
}

// Write L_kk (lower, zero above) and inv(L_kk) as FP32.
template <typename T>
__global__ void k_potrf_store(const T *__restrict__ W, const T *__restrict__ Winv,
                              const T *__restrict__ Dinv, float *__restrict__ Akk,
                              float *__restrict__ Linv, int nb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * nb) return;
  const int r = (int)(e / nb), c = (int)(e % nb);
  const int a = r / BS, b = c / BS;
  Akk[e] = (c <= r) ? (float)W[e] : 0.0f;
  T v = (T)0;
  if (a == b)
    v = Dinv[(int64_t)a * BS * BS + (r % BS) * BS + (c % BS)];
  else if (a > b)
    v = Winv[e];
  Linv[e] = (float)v;
}

template <typename T>
static void potrf_tile_t(float *Akk, float *Linv, int k, const TileLayout &L, FactorWork &w,
                         hipStream_t s) {
  const int nb = L.nb, NB = nb / BS;
  T *W = (T *)w.W64, *Winv = (T *)w.Winv64, *Dinv = (T *)w.Dinv64;
  const unsigned eb = (unsigned)(((int64_t)nb * nb + 255) / 256);
  const int64_t colbase = (int64_t)k * nb;
  hipLaunchKernelGGL(k_potrf_load<T>, dim3(eb), dim3(256), 0, s, Akk, W, nb);
  for (int st = 0; st < NB; ++st) {
    hipLaunchKernelGGL(k_potrf_diag64<T>, dim3(1), dim3(64), 0, s, W, nb, st, Dinv, w.flag,
                       colbase);
    const int rest = NB - 1 - st;
    if (rest > 0) {
      hipLaunchKernelGGL(k_potrf_trsm64<T>, dim3(rest), dim3(256), 0, s, W, nb, st, Dinv);
      hipLaunchKernelGGL(k_potrf_syrk64<T>, dim3(rest * (rest + 1) / 2), dim3(256), 0, s, W, nb,
                         st);
    }
  }
  for (int delta = 1; delta < NB; ++delta)
    hipLaunchKernelGGL(k_trtri_off64<T>, dim3(NB - delta), dim3(256), 0, s, W, Winv, nb, delta,
                       Dinv);
  hipLaunchKernelGGL(k_potrf_store<T>, dim3(eb), dim3(256), 0, s, W, Winv, Dinv, Akk, Linv, nb);
}

void launch_potrf_tile(float *Akk, float *Linv, int k, const TileLayout &L, bool fp64,
                       FactorWork &w, hipStream_t s) {
  if (fp64)
    potrf_tile_t<double>(Akk, Linv, k, L, w, s);
  else
    potrf_tile_t<float>(Akk, Linv, k, L, w, s);
}

// ---------------------------------------------------------------------------
// Panel TRSM as an FP32 MFMA product: P_i = A_ik * inv(L_kk)^T, i > k.  The
// output goes to the panel buffer (A_ik is read by other workgroups of the
// same tile).  Each 128 x 128 block also leaves its FP64 sum of squares and
// its max |entry| for the operand norms and scales.
constexpr int UB = 128;  // block edge of the factorization GEMMs
typedef GemmShape<UB, UB, 2, 2> UpdShape;

__global__ __launch_bounds__(256) void k_trsm_panel(const float *__restrict__ Astore,
                                                    const float *__restrict__ Linv, int k, int nb,
                                                    int SB, float *__restrict__ P32,
                                                    double *__restrict__ pnorm_part,
                                                    float *__restrict__ pmax_part) {
  typedef UpdShape S;
  __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];
  __shared__ double shd[4];
  __shared__ float shf[4];
  const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int nsub = SB * SB;
  const int sub = (int)(bid % nsub);
  const int64_t t = bid / nsub;
  const int64_t i = k + 1 + t;
  const int si = sub / SB, sj = sub % SB;
  const int64_t te = (int64_t)nb * nb;
  const float *Ablk = Astore + (i * (i + 1) / 2 + k) * te + (int64_t)si * UB * nb;
  const float *Bblk = Linv + (int64_t)sj * UB * nb;
  const int64_t kbytes = (int64_t)min(nb, (sj + 1) * UB) * 4;  // inv(L) is lower triangular
  OpF32::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  gemm_nt_core<OpF32, S>(OpF32{}, (const uint8_t *)Ablk, (int64_t)nb * 4, UB, (const uint8_t *)Bblk,
                         (int64_t)nb * 4, UB, kbytes, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float *out = P32 + t * te + (int64_t)si * UB * nb + sj * UB;
  double ss = 0.0;
  float mx = 0.0f;
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = S::row(wave, tm, e, lane);
        const int c = S::col(wave, tn, lane);
        const float v = acc[tm][tn][e];
        out[(int64_t)r * nb + c] = v;
        ss += (double)v * (double)v;
        mx = fmaxf(mx, fabsf(v));
      }
  ss = block_sum<4>(ss, shd);
  mx = block_max<4>(mx, shf);
  if (threadIdx.x == 0) {
    pnorm_part[bid] = ss;
    pmax_part[bid] = mx;
  }
}

void launch_trsm_panel(const float *Astore, const float *Linv, int k, const TileLayout &L,
                       FactorWork &w, const PanelBuf &pb, hipStream_t s) {
  const int SB = L.nb / UB;
  const int64_t tiles = L.nt - 1 - k;
  if (tiles <= 0) return;
  hipLaunchKernelGGL(k_trsm_panel, dim3((unsigned)(tiles * SB * SB)), dim3(256), 0, s, Astore,
                     Linv, k, L.nb, SB, pb.P32, w.pnorm_part, w.pmax_part);
}

// Panel conversion: reduce each tile's partial norms (fixed order), pick the
// FP8 power-of-two scale, copy the FP32 L_ik into the factor storage and
// write the FP16 copy (unscaled) and the scaled FP8 E4M3 copy.
constexpr int CONV_CHUNK = 4096;  // elements per workgroup

__global__ __launch_bounds__(256) void k_convert_panel(
    const float *__restrict__ P32, float *__restrict__ Astore, _Float16 *__restrict__ P16,
    uint8_t *__restrict__ P8, const double *__restrict__ pnorm_part,
    const float *__restrict__ pmax_part, int parts, float *__restrict__ pnorm,
    int *__restrict__ pexp8, int k, int nb, int chunks, int need16, int need8) {
  const int64_t t = blockIdx.x / chunks;
  const int ch = blockIdx.x % chunks;
  const int64_t i = k + 1 + t;
  double ss = 0.0;
  float mx = 0.0f;
  for (int q = 0; q < parts; ++q) {
    ss += pnorm_part[t * parts + q];
    mx = fmaxf(mx, pmax_part[t * parts + q]);
  }
  const float s8 = pow2_scale(mx, 448.0f);
  const int64_t te = (int64_t)nb * nb;
  const float *src = P32 + t * te;
  float *dstL = Astore + (i * (i + 1) / 2 + k) * te;
  const int64_t e0 = (int64_t)ch * CONV_CHUNK;
  for (int64_t e = e0 + threadIdx.x * 4; e < e0 + CONV_CHUNK; e += 256 * 4) {
    const float4 v = *(const float4 *)(src + e);
    *(float4 *)(dstL + e) = v;
    if (need16) {
      typedef _Float16 h4 __attribute__((ext_vector_type(4)));
      h4 h = {(_Float16)v.x, (_Float16)v.y, (_Float16)v.z, (_Float16)v.w};
      *(h4 *)(P16 + t * te + e) = h;
    }
    if (need8) {
      const uint32_t q = (uint32_t)f32_to_e4m3(v.x * s8) | ((uint32_t)f32_to_e4m3(v.y * s8) << 8) |
                         ((uint32_t)f32_to_e4m3(v.z * s8) << 16) |
                         ((uint32_t)f32_to_e4m3(v.w * s8) << 24);
      *(uint32_t *)(P8 + t * te + e) = q;
    }
  }
  if (ch == 0 && threadIdx.x == 0) {
    pnorm[t] = (float)sqrt(ss);
    pexp8[t] = ilogbf(s8);  // s8 = 2^pexp8
  }
}

void launch_convert_panel(float *Astore, int k, const TileLayout &L, FactorWork &w,
                          const PanelBuf &pb, bool need16, bool need8, hipStream_t s) {
  const int64_t tiles = L.nt - 1 - k;
  if (tiles <= 0) return;
  const int chunks = (int)((int64_t)L.nb * L.nb / CONV_CHUNK);
  const int SB = L.nb / UB;
  hipLaunchKernelGGL(k_convert_panel, dim3((unsigned)(tiles * chunks)), dim3(256), 0, s, pb.P32,
                     Astore, pb.P16, pb.P8, w.pnorm_part, w.pmax_part, SB * SB, pb.pnorm, pb.pexp8,
                     k, L.nb, chunks, need16 ? 1 : 0, need8 ? 1 : 0);
}

// Trailing update by a group of consecutive panels k0 .. k0+npan-1:
//   A_ij -= sum_k L_ik L_jk^T   for the tiles (i, j), jlo <= j <= jhi, j <= i < NT,
// one 128 x 128 block per workgroup, FP32 accumulation over all panels of
// the group (the FP32 block of C is read and written once per group).  The
// operand precision is chosen per (tile, panel), uniform across the
// workgroup:
//   FP32 on diagonal tiles, on panels k < high_panels and under the FP32 policy;
//   FIXED: fixed_prec; ADAPTIVE: lowest allowed p with
//   u_p ||L_ik||_F ||L_jk||_F <= thr (= eps ||A||_F / NT).
struct PanelSet {
  const float *P32[KRR_MAX_GROUP];
  const _Float16 *P16[KRR_MAX_GROUP];
  const uint8_t *P8[KRR_MAX_GROUP];
  const float *pnorm[KRR_MAX_GROUP];
  const int *pexp8[KRR_MAX_GROUP];
};

__global__ __launch_bounds__(256) void k_update(float *__restrict__ Astore, PanelSet ps, int k0,
                                                int npan, int jlo, int jhi, int NT, int nb, int SB,
                                                int mode, int allow16, int allow8, int high_panels,
                                                int fixed_prec, double thr,
                                                unsigned long long *counts, uint8_t *pmap,
                                                int64_t ntiles_all) {
  typedef UpdShape S;
  __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];
  const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int nsub = SB * SB;
  const int sub = (int)(bid % nsub);
  int64_t tt = bid / nsub;
  int64_t i, j;
  if (jhi == NT - 1) {  // triangle of all tiles right of column jlo
    int ta, tb;
    tri_decode(tt, ta, tb);
    i = jlo + ta;
    j = jlo + tb;
  } else {  // a few columns: walk them
    j = jlo;
    while (tt >= NT - j) {
      tt -= NT - j;
      ++j;
    }
    i = j + tt;
  }
  const int si = sub / SB, sj = sub % SB;
  const int64_t te = (int64_t)nb * nb;

  auto choose = [&](int q) {
    const int k = k0 + q;
    const int64_t a = i - k - 1, b = j - k - 1;
    int prec = KRR_PREC_FP32;
    if (i != j && k >= high_panels) {
      if (mode == KRR_POLICY_FIXED) {
        prec = fixed_prec;
      } else if (mode == KRR_POLICY_ADAPTIVE) {
        const double prod = (double)ps.pnorm[q][a] * (double)ps.pnorm[q][b];
        if (allow8 && 0.0625 * prod <= thr)
          prec = KRR_PREC_FP8;
        else if (allow16 && 0.00048828125 * prod <= thr)
          prec = KRR_PREC_FP16;
      }
    }
    return prec;
  };
  // One pass per operand type (FP32 panels, then FP16, then FP8), so each
  // MFMA flavour is instantiated once and the shared accumulator stays put.
  OpF32::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  for (int q = 0; q < npan; ++q) {
    if (choose(q) != KRR_PREC_FP32) continue;
    const int64_t a = i - (k0 + q) - 1, b = j - (k0 + q) - 1;
    gemm_nt_core<OpF32, S>(OpF32{}, (const uint8_t *)(ps.P32[q] + a * te + (int64_t)si * UB * nb),
                           (int64_t)nb * 4, UB,
                           (const uint8_t *)(ps.P32[q] + b * te + (int64_t)sj * UB * nb),
                           (int64_t)nb * 4, UB, (int64_t)nb * 4, acc, lds);
  }
  for (int q = 0; q < npan; ++q) {
    if (choose(q) != KRR_PREC_FP16) continue;
    const int64_t a = i - (k0 + q) - 1, b = j - (k0 + q) - 1;
    gemm_nt_core<OpF16, S>(OpF16{}, (const uint8_t *)(ps.P16[q] + a * te + (int64_t)si * UB * nb),
                           (int64_t)nb * 2, UB,
                           (const uint8_t *)(ps.P16[q] + b * te + (int64_t)sj * UB * nb),
                           (int64_t)nb * 2, UB, (int64_t)nb * 2, acc, lds);
  }
  for (int q = 0; q < npan; ++q) {
    if (choose(q) != KRR_PREC_FP8) continue;
    const int64_t a = i - (k0 + q) - 1, b = j - (k0 + q) - 1;
    OpF8 op;
    op.sa = 127 - ps.pexp8[q][a];
    op.sb = 127 - ps.pexp8[q][b];
    gemm_nt_core<OpF8, S>(op, ps.P8[q] + a * te + (int64_t)si * UB * nb, nb, UB,
                          ps.P8[q] + b * te + (int64_t)sj * UB * nb, nb, UB, nb, acc, lds);
  }
  if (sub == 0 && threadIdx.x == 0) {
    for (int q = 0; q < npan; ++q) {
      const int prec = choose(q);
      atomicAdd(&counts[prec], 1ULL);
      if (pmap) pmap[(int64_t)(k0 + q) * ntiles_all + i * (i + 1) / 2 + j] = (uint8_t)prec;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float *C = Astore + (i * (i + 1) / 2 + j) * te + (int64_t)si * UB * nb + sj * UB;
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = S::row(wave, tm, e, lane);
        const int c = S::col(wave, tn, lane);
        C[(int64_t)r * nb + c] -= acc[tm][tn][e];
      }
}

void launch_update(float *Astore, int k0, int npan, int jlo, int jhi, const TileLayout &L,
                   const UpdatePolicy &pol, FactorWork &w, const PanelBuf *const *pbs,
                   uint8_t *pmap, hipStream_t s) {
  const int NT = L.nt;
  if (npan <= 0 || jlo > jhi || jlo >= NT) return;
  if (jhi > NT - 1) jhi = NT - 1;
  int64_t tiles = 0;
  if (jhi == NT - 1) {
    const int64_t T = NT - jlo;
    tiles = T * (T + 1) / 2;
  } else {
    for (int j = jlo; j <= jhi; ++j) tiles += NT - j;
  }
  PanelSet ps{};
  for (int q = 0; q < npan; ++q) {
    ps.P32[q] = pbs[q]->P32;
    ps.P16[q] = pbs[q]->P16;
    ps.P8[q] = pbs[q]->P8;
    ps.pnorm[q] = pbs[q]->pnorm;
    ps.pexp8[q] = pbs[q]->pexp8;
  }
  const int SB = L.nb / UB;
  const int64_t blocks = tiles * SB * SB;
  hipLaunchKernelGGL(k_update, dim3((unsigned)blocks), dim3(256), 0, s, Astore, ps, k0, npan, jlo,
                     jhi, NT, L.nb, SB, pol.mode, pol.allow16, pol.allow8, pol.high_panels,
                     pol.fixed_prec, pol.thr, w.counts, pmap, L.ntiles());
}

// Test hook: the factorization's FP8 encoder applied elementwise.
__global__ void k_encode_fp8(const float *__restrict__ x, int64_t n, uint8_t *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = f32_to_e4m3(x[e]);
}

void launch_encode_fp8(const float *x, int64_t n, uint8_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_encode_fp8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, out);
}

}  // namespace krr
