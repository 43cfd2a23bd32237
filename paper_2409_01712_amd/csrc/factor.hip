// Associate phase, first half: tile Cholesky of K + lambda*I with a
// per-update choice of operand precision (arXiv 2409.01712, Algorithm 3;
// "Deploying a Four-Precision Cholesky-Based Solver").
//
// Right-looking over panels k = 0 .. NT-1:
//   POTRF   L_kk = chol(A_kk) in FP64 (or FP32 on the plain path) by 64-column
//           steps, with the inverses of its 64 x 64 diagonal blocks, and
//           L_kk^{-1} formed from them;
//   TRSM    L_ik = A_ik L_kk^{-T}: by block substitution with L_kk (the row
//           tile on the critical path) or as an FP32 MFMA product with
//           L_kk^{-1} (the rest);
//   convert L_ik to FP16 / FP8 E4M3 copies with a per-tile power-of-two
//           scale (produced once per panel, consumed by every update);
//   update  A_ij -= L_ik L_jk^T for k < j <= i: FP32 on diagonal tiles and
//           early panels, otherwise FP16 or FP8 operands chosen per update
//           from the operand tile norms, always accumulated in FP32.
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "internal.h"

namespace krr {

constexpr int BS = 64;  // sub-block of the diagonal-tile factorization

// ---------------------------------------------------------------------------
// Diagonal tile: blocked Cholesky and triangular inverse, 64 x 64 sub-blocks.
// W holds the nb x nb tile (row-major) in T = double or float.


// 64 x 64 block products on 16 x 16 x 4 MFMA tiles (FP64 or FP32): wave w
// computes rows 16w .. 16w+15 of C = A op(B) for all 64 columns.  A, B are
// [64][BS + 1] LDS arrays; op(B)[k][j] = B[j][k] if BT else B[k][j].
// acc[ct] holds C rows (layout of the MFMA type), columns 16 ct + l % 16.
template <typename T> struct M16;
template <> struct M16<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  KRR_DEV static v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  KRR_DEV static int row(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <> struct M16<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  KRR_DEV static v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  KRR_DEV static int row(int r, int lane) { return 4 * (lane >> 4) + r; }
};

// Value of v held by lane src (wave-uniform), broadcast to the wave.
KRR_DEV double bcast(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
KRR_DEV float bcast(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}

// 1 / sqrt(x): hardware estimate refined by two Newton-Raphson steps
// y <- y + (y / 2)(1 - x y^2), each of which doubles the correct bits.
KRR_DEV double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double h = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, h, y);
  }
  return y;
}
KRR_DEV float rsqrt_nr(float x) { return 1.0f / sqrtf(x); }

// LDS reads after LDS writes of other lanes of the same wave: the wave's LDS
// operations complete in order, so only the compiler must be kept in order.
KRR_DEV void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16 x 16 Cholesky factor of the diagonal block at (b, b) of S, in place
// (one wave; lane li holds row li, lanes 16..63 mirror lanes 0..15), by
// 4-column blocks c = 0, 4, 8, 12:
//   columns c .. c+3 of every row in registers, factored column by column:
//   the pivot of lane c+j broadcast, l = column c+j of L, and the updates of
//   the block's later columns with l_k broadcast from lane k; the next pivot
//   is lane c+j+1's own updated diagonal, so the chain from one pivot to the
//   next is one FMA and one broadcast;
//   then the rank-4 update of the trailing rows and columns by one
//   16 x 16 x 4 MFMA (the rest of the block is left as it is).
// L goes to the lower triangle of the block (zeros above it); rv[j] =
// 1 / L_jj; badj: first column with a non-positive pivot (replaced by 1
// there), or -1.
template <typename T>
KRR_DEV void chol16(T (*S)[BS + 1], int b, T (&rv)[16], int &badj) {
  typedef typename M16<T>::v4 v4;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  badj = -1;
#pragma unroll
  for (int c = 0; c < 16; c += 4) {
    T d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = S[b + li][b + c + q];
    T pivn = bcast(d[0], c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      T piv = pivn;
      const bool bad = !(piv > (T)0);
      badj = (bad && badj < 0) ? c + j : badj;
      piv = bad ? (T)1 : piv;
      const T r = rsqrt_nr(piv);
      rv[c + j] = r;
      const T l = (li == c + j) ? piv * r : d[j] * r;
      d[j] = l;
      if (j < 3) {
        pivn = bcast(d[j + 1] - l * l, c + j + 1);
#pragma unroll
        for (int k = j + 1; k < 4; ++k) d[k] -= l * bcast(l, c + k);
      }
    }
    if (lane < 16) {
#pragma unroll
      for (int q = 0; q < 4; ++q) S[b + li][b + c + q] = (c + q <= li) ? d[q] : (T)0;
    }
    if (c < 12) {
      wave_lds_sync();
      // S_ij -= sum_t L_i,c+t L_j,c+t for i, j >= c + 4
      const T lv = S[b + li][b + c + lg];
      v4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = S[b + M16<T>::row(r, lane)][b + li];
      acc = M16<T>::mma(-lv, lv, acc);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = M16<T>::row(r, lane);
        if (row >= c + 4 && li >= c + 4) S[b + row][b + li] = acc[r];
      }
      wave_lds_sync();
    }
  }
}

// Factor the 16 x 16 diagonal block b of S (one wave, all lanes): L into S
// (zero above the diagonal), its inverse into X (lane li computes column li
// by forward substitution with the L entries read back from LDS).
template <typename T>
KRR_DEV void diag16(T (*S)[BS + 1], T (*X)[BS + 1], int b, int32_t *flag, int64_t col0) {
  const int lane = threadIdx.x & 63, li = lane & 15;
  T rv[16];
  int badj;
  chol16<T>(S, b, rv, badj);
  if (badj >= 0 && lane == 0) atomicCAS(flag, 0, (int32_t)(col0 + b + badj + 1));
  wave_lds_sync();
  // column li of inv(L_bb): x_q = (e_li - sum_{p<q} L_qp x_p)_q / L_qq,
  // row q of L read as a contiguous (broadcast) run, the sum in p order
  T x[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    T acc = (q == li) ? (T)1 : (T)0;
#pragma unroll
    for (int p = 0; p < q; ++p) acc -= S[b + q][b + p] * x[p];
    x[q] = acc * rv[q];
  }
  if (lane < 16) {
#pragma unroll
    for (int q = 0; q < 16; ++q) X[b + q][b + li] = x[q];
  }
}

// S_ib,jb -= L_ib,kb L_jb,kb^T (16 x 16 blocks of S, one wave).
template <typename T>
KRR_DEV void upd16(T (*S)[BS + 1], int ib, int jb, int kb) {
  typedef typename M16<T>::v4 v4;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4, b = 16 * kb;
  v4 acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = S[16 * ib + M16<T>::row(r, lane)][16 * jb + li];
#pragma unroll
  for (int k0 = 0; k0 < 16; k0 += 4)
    acc = M16<T>::mma(-S[16 * ib + li][b + k0 + lg], S[16 * jb + li][b + k0 + lg], acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) S[16 * ib + M16<T>::row(r, lane)][16 * jb + li] = acc[r];
}

// X_ib,jb = -inv(L_ib,ib) sum_{kb=jb}^{ib-1} L_ib,kb X_kb,jb (one wave), the
// sum staged in the output block.
template <typename T>
KRR_DEV void inv16(const T (*S)[BS + 1], T (*X)[BS + 1], int ib, int jb) {
  typedef typename M16<T>::v4 v4;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  v4 acc = {0, 0, 0, 0};
  for (int kb = jb; kb < ib; ++kb)
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4)
      acc = M16<T>::mma(S[16 * ib + li][16 * kb + k0 + lg], X[16 * kb + k0 + lg][16 * jb + li], acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) X[16 * ib + M16<T>::row(r, lane)][16 * jb + li] = acc[r];
  wave_lds_sync();
  T bv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bv[r] = X[16 * ib + 4 * r + lg][16 * jb + li];
  v4 out = {0, 0, 0, 0};
#pragma unroll
  for (int r = 0; r < 4; ++r) out = M16<T>::mma(-X[16 * ib + li][16 * ib + 4 * r + lg], bv[r], out);
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < 4; ++r) X[16 * ib + M16<T>::row(r, lane)][16 * jb + li] = out[r];
}

// Factor sub-block (s, s) of the tile and invert it, one workgroup of four
// waves, blocked by 16 columns (blocks kb = 0..3).  Wave 0 carries the
// chain from one diagonal block to the next:
//   panel   L_ib,kb = A_ib,kb inv(L_kb,kb)^T      (wave ib-kb-1, one per block)
//   --- barrier ---
//   wave 0: A_kb+1,kb+1 -= L L^T, then the 16 x 16 factor and inverse of it;
//   waves 1..3 meanwhile: the other updates A_ib,jb -= L_ib,kb L_jb,kb^T
//   (kb < jb <= ib) and the completed inverse blocks of row kb,
//   X_kb,jb = -inv(L_kb,kb) sum_{p=jb}^{kb-1} L_kb,p X_p,jb
//   --- barrier ---
// so each 16-column step takes two barriers and the next diagonal factor
// overlaps the rest of the step.  Every block gets the same products in the
// same order as in the plain blocked algorithm.
template <typename T>
KRR_DEV void diag64_body(T (*S)[BS + 1], T (*X)[BS + 1], int32_t *flag, int64_t col0) {
  typedef typename M16<T>::v4 v4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  if (wave == 0) diag16<T>(S, X, 0, flag, col0);
  __syncthreads();
  for (int kb = 0; kb < 4; ++kb) {
    const int b = 16 * kb;
    if (kb < 3) {
      const int ib = kb + 1 + wave;
      if (ib < 4) {
        v4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4)
          acc = M16<T>::mma(S[16 * ib + li][b + k0 + lg], X[b + li][b + k0 + lg], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) S[16 * ib + M16<T>::row(r, lane)][b + li] = acc[r];
      }
      __syncthreads();
    }
    if (wave == 0) {
      if (kb < 3) {
        upd16<T>(S, kb + 1, kb + 1, kb);
        wave_lds_sync();
        diag16<T>(S, X, 16 * (kb + 1), flag, col0);
      }
    } else {
      // pairs (ib, jb), kb < jb <= ib < 4, other than (kb+1, kb+1), then
      // the inverse blocks (kb, jb), jb < kb, dealt over waves 1..3
      int item = 0;
      for (int jb = kb + 1; jb < 4; ++jb)
        for (int ib = jb; ib < 4; ++ib) {
          if (ib == kb + 1 && jb == kb + 1) continue;
          if (item++ % 3 == wave - 1) upd16<T>(S, ib, jb, kb);
        }
      for (int jb = 0; jb < kb; ++jb)
        if (item++ % 3 == wave - 1) inv16<T>(S, X, kb, jb);
    }
    __syncthreads();
  }
}

// Write L (zero above the diagonal) and inv(L) of a factored 64 x 64 block;
// Lf, If (or null): FP32 copies of both at the block's place in FP32 tiles
// (leading dimension ld).
template <typename T>
__device__ __forceinline__ void diag64_store(const T (*S)[BS + 1], const T (*X)[BS + 1], T *Lblk,
                                             int64_t ld, T *Dblk, float *Lf = nullptr,
                                             float *If = nullptr) {
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = threadIdx.x + 256 * q, r = e / BS, c = e % BS;
    const T l = (c <= r) ? S[r][c] : (T)0, x = (c <= r) ? X[r][c] : (T)0;
    Lblk[(int64_t)r * ld + c] = l;
    Dblk[e] = x;
    if (Lf) Lf[(int64_t)r * ld + c] = (float)l;
    if (If) If[(int64_t)r * ld + c] = (float)x;
  }
}

// First diagonal block of the tile: W_00 -> L_00 (in WL) and inv(L_00).
template <typename T>
KRR_DEV void potrf_diag64_first(const T *__restrict__ W, T *__restrict__ WL, int nb,
                                T *__restrict__ Dinv, int32_t *flag, int64_t colbase,
                                float *Lf = nullptr, float *If = nullptr) {
  __shared__ T S[BS][BS + 1];  // the block, overwritten by L
  __shared__ T X[BS][BS + 1];  // inv(L)
  {
    T v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + 256 * q, r = e / BS, c = e % BS;
      v[q] = (c <= r) ? W[(int64_t)r * nb + c] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = threadIdx.x + 256 * q;
      S[e / BS][e % BS] = v[q];
    }
  }
  __syncthreads();
  diag64_body<T>(S, X, flag, colbase);
  diag64_store<T>(S, X, WL, nb, Dinv, Lf, If);
}

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_diag64(const T *__restrict__ W, T *__restrict__ WL,
                                                      int nb, T *__restrict__ Dinv, int32_t *flag,
                                                      int64_t colbase, float *Lf, float *If) {
  potrf_diag64_first<T>(W, WL, nb, Dinv, flag, colbase, Lf, If);
}

template <typename T, bool BT>
__device__ __forceinline__ void mm64(const T (*A)[BS + 1], const T (*B)[BS + 1],
                                     typename M16<T>::v4 (&acc)[4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < BS; k0 += 4) {
    const T av = A[16 * wave + li][k0 + lg];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const T bv = BT ? B[16 * ct + li][k0 + lg] : B[k0 + lg][16 * ct + li];
      acc[ct] = M16<T>::mma(av, bv, acc[ct]);
    }
  }
}

template <typename T>
__device__ __forceinline__ void zero4(typename M16<T>::v4 (&acc)[4]) {
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = (typename M16<T>::v4){0, 0, 0, 0};
}

// dst (ld) = alpha * acc, or dst += alpha * acc when ADD
template <typename T, bool ADD>
__device__ __forceinline__ void store64(T *dst, int64_t ld, const typename M16<T>::v4 (&acc)[4],
                                        T alpha) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // ADD: all sixteen loads issued before the first store (the compiler may
  // not move a load past a store to a possibly equal address)
  T old[4][4] = {};
  if (ADD) {
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        old[ct][r] = dst[(int64_t)(16 * wave + M16<T>::row(r, lane)) * ld + 16 * ct + (lane & 15)];
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      T *p = dst + (int64_t)(16 * wave + M16<T>::row(r, lane)) * ld + 16 * ct + (lane & 15);
      *p = ADD ? old[ct][r] + alpha * acc[ct][r] : alpha * acc[ct][r];
    }
}

// dst (ld, FP32) = alpha * acc
template <typename T>
__device__ __forceinline__ void store64f(float *dst, int64_t ld, const typename M16<T>::v4 (&acc)[4],
                                         T alpha) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      dst[(int64_t)(16 * wave + M16<T>::row(r, lane)) * ld + 16 * ct + (lane & 15)] =
          (float)(alpha * acc[ct][r]);
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

// acc (layout of mm64) into a 64 x 64 LDS block.
template <typename T>
__device__ __forceinline__ void store_lds64(T (*dst)[BS + 1], const typename M16<T>::v4 (&acc)[4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) dst[16 * wave + M16<T>::row(r, lane)][16 * ct + (lane & 15)] = acc[ct][r];
}

// Step s of the tile factorization, one workgroup per block pair (a, b) with
// s < b <= a < nb / 64:
//   P_a = W_as inv(L_ss)^T   (block (a, s) of L; written by the pair (a, a)),
//   W_ab -= P_a P_b^T,
// and the pair (s+1, s+1) goes on to factor its updated block -- the next
// diagonal step -- without writing it back.  Block column s of W is only
// read in this step (the factor goes to WL), so the pairs need no ordering.
//
// With Winv (the tile's FP64 inverse, leading dimension nb), the workgroups
// bid >= npairs build inv(L_kk) = X a block row at a time, its sums
//   X_st = -inv(L_ss) sum_{p=t}^{s-1} L_sp X_pt   (X_tt = inv(L_tt) from Dinv)
// accumulated in Winv as the rows become final, one product per workgroup
// and step:
//   finalize (extra < s): X_st = -inv(L_ss) (S_st + L_s,s-1 X_s-1,t), S_st the
//     sum over p < s - 1 kept in Winv (none when t = s - 1);
//   accumulate (the rest): S_rt += L_r,s-1 X_s-1,t for the later rows
//     r > s and t < s (written, not added, when t = s - 1: the first term).
// Each sum is formed in increasing p, one MFMA product per term as in a
// single accumulator.  If (or null): the FP32 inverse tile gets the final
// blocks.  Lf (or null): the FP32 factor tile gets the panel blocks and the
// next diagonal block as they are written.
template <typename T>
KRR_DEV void load_acc64(const T *src, int64_t ld, typename M16<T>::v4 (&acc)[4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc[ct][r] = src[(int64_t)(16 * wave + M16<T>::row(r, lane)) * ld + 16 * ct + (lane & 15)];
}

// Device view of a RowPanel (WX in T); final: the launch after the last
// step (one workgroup per block row, the last block column alone).
template <typename T>
struct RowPanelDev {
  const float *A;
  T *WX;
  float *P32;
  double *pnorm_part;
  float *pmax_part;
  int parts, final_launch;
};

template <typename T>
KRR_DEV void potrf_step_body(T *__restrict__ W, T *__restrict__ WL, int nb, int s,
                             T *__restrict__ Dinv, int32_t *flag, int64_t colbase, int bid,
                             int npairs = 1 << 30, T *__restrict__ Winv = nullptr,
                             float *Lf = nullptr, float *If = nullptr, int ninv = 1 << 29,
                             const RowPanelDev<T> *rp = nullptr) {
  typedef typename M16<T>::v4 v4;
  __shared__ T buf[3][BS][BS + 1];
  if (rp && bid >= npairs + ninv) {
    // The next row tile's panel, block column s: workgroup (x, b) forms
    // L_x,s = WX_x,s inv(L_ss)^T and L_b,s, subtracts L_x,s L_b,s^T from
    // WX_x,b (b > s; at s = 0 WX starts from A), and for b = s + 1 writes
    // L_x,s out; after the last step, workgroup x forms L_x,NB-1 alone.
    const int NB = nb / BS, e = bid - npairs - ninv;
    __shared__ double shd[4];
    __shared__ float shf[4];
    const int x = rp->final_launch ? e : e / (NB - 1 - s);
    const int b = rp->final_launch ? s : s + 1 + e % (NB - 1 - s);
    T(*Xa)[BS + 1] = buf[0];
    T(*Xb)[BS + 1] = buf[1];
    T(*Li)[BS + 1] = buf[2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t oxs = (int64_t)(x * BS) * nb + s * BS, oxb = (int64_t)(x * BS) * nb + b * BS;
    if (s == 0) {
      for (int q = threadIdx.x; q < BS * BS; q += 256)
        Xa[q / BS][q % BS] = (T)rp->A[oxs + (int64_t)(q / BS) * nb + q % BS];
    } else {
      load64(Xa, rp->WX + oxs, nb);
    }
    load64(Li, Dinv + (int64_t)s * BS * BS, BS);
    if (!rp->final_launch) load64(Xb, W + (int64_t)(b * BS) * nb + s * BS, nb);
    __syncthreads();
    v4 pa[4], pb[4];
    zero4<T>(pa);
    mm64<T, true>(Xa, Li, pa);
    if (!rp->final_launch) {
      zero4<T>(pb);
      mm64<T, true>(Xb, Li, pb);
      __syncthreads();
      store_lds64<T>(Xa, pa);
      store_lds64<T>(Xb, pb);
      __syncthreads();
      v4 acc[4];
      zero4<T>(acc);
      mm64<T, true>(Xa, Xb, acc);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t o = oxb + (int64_t)(16 * wave + M16<T>::row(r, lane)) * nb + 16 * ct +
                            (lane & 15);
          const T prev = s == 0 ? (T)rp->A[o] : rp->WX[o];
          rp->WX[o] = prev - acc[ct][r];
        }
    }
    if (rp->final_launch || b == s + 1) {  // L_x,s out, with its sum of squares and maximum
      double ss = 0.0;
      float mx = 0.0f;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float f = (float)pa[ct][r];
          rp->P32[oxs + (int64_t)(16 * wave + M16<T>::row(r, lane)) * nb + 16 * ct + (lane & 15)] =
              f;
          ss += (double)f * (double)f;
          mx = fmaxf(mx, fabsf(f));
        }
      ss = block_sum<4>(ss, shd);
      mx = block_max<4>(mx, shf);
      if (threadIdx.x == 0) {
        rp->pnorm_part[x * NB + s] = ss;
        rp->pmax_part[x * NB + s] = mx;
      }
    }
    return;
  }
  if (bid >= npairs) {
    const int extra = bid - npairs, p = s - 1;
    int r, t;
    bool fin;
    if (extra < s) {
      fin = true;
      r = s;
      t = extra;
    } else {
      fin = false;
      r = s + 1 + (extra - s) / s;
      t = (extra - s) % s;
    }
    T(*Ab)[BS + 1] = buf[0];
    T(*Bb)[BS + 1] = buf[1];
    T(*Cb)[BS + 1] = buf[2];
    T *Srt = Winv + (int64_t)(r * BS) * nb + t * BS;
    v4 acc[4];
    if (t < p) load_acc64<T>(Srt, nb, acc);  // the terms p' < s - 1 so far
    else zero4<T>(acc);
    // + L_r,s-1 X_s-1,t
    load64(Ab, WL + (int64_t)(r * BS) * nb + p * BS, nb);
    if (t == p) load64(Bb, Dinv + (int64_t)p * BS * BS, BS);
    else load64(Bb, Winv + (int64_t)(p * BS) * nb + t * BS, nb);
    __syncthreads();
    mm64<T, false>(Ab, Bb, acc);
    if (!fin) {
      store64<T, false>(Srt, nb, acc, (T)1);
      return;
    }
    __syncthreads();
    store_lds64<T>(Cb, acc);
    load64(Ab, Dinv + (int64_t)s * BS * BS, BS);
    __syncthreads();
    v4 out[4];
    zero4<T>(out);
    mm64<T, false>(Ab, Cb, out);
    store64<T, false>(Srt, nb, out, (T)-1);
    if (If) store64f<T>(If + (int64_t)(r * BS) * nb + t * BS, nb, out, (T)-1);
    return;
  }
  int a, b;
  tri_decode(bid, a, b);
  a += s + 1;
  b += s + 1;
  T(*Xa)[BS + 1] = buf[0];
  T(*Xb)[BS + 1] = buf[1];
  T(*Li)[BS + 1] = buf[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T *Wab = W + (int64_t)(a * BS) * nb + b * BS;
  const bool diag = a == s + 1 && b == s + 1;
  // the next diagonal block's entries, loaded with the operands so that
  // their latency is not on the path to its factorization
  T wv[4][4];
  if (diag) {
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * wave + M16<T>::row(r, lane), col = 16 * ct + (lane & 15);
        wv[ct][r] = (col <= row) ? Wab[(int64_t)row * nb + col] : (T)0;
      }
  }
  load64(Xa, W + (int64_t)(a * BS) * nb + s * BS, nb);
  load64(Li, Dinv + (int64_t)s * BS * BS, BS);
  if (a != b) load64(Xb, W + (int64_t)(b * BS) * nb + s * BS, nb);
  __syncthreads();
  v4 pa[4], pb[4];
  zero4<T>(pa);
  mm64<T, true>(Xa, Li, pa);
  if (a != b) {
    zero4<T>(pb);
    mm64<T, true>(Xb, Li, pb);
  }
  __syncthreads();
  store_lds64<T>(Xa, pa);
  if (a != b) store_lds64<T>(Xb, pb);
  else {
    store64<T, false>(WL + (int64_t)(a * BS) * nb + s * BS, nb, pa, (T)1);
    if (Lf) store64f<T>(Lf + (int64_t)(a * BS) * nb + s * BS, nb, pa, (T)1);
  }
  __syncthreads();
  v4 acc[4];
  zero4<T>(acc);
  mm64<T, true>(Xa, a == b ? Xa : Xb, acc);
  if (diag) {
    // buf[2] (inv(L_ss)) and buf[1] (unused: a == b) take the next block
    T(*S)[BS + 1] = buf[2];
    T(*X)[BS + 1] = buf[1];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * wave + M16<T>::row(r, lane), col = 16 * ct + (lane & 15);
        S[row][col] = (col <= row) ? wv[ct][r] - acc[ct][r] : (T)0;
      }
    __syncthreads();
    diag64_body<T>(S, X, flag, colbase + (int64_t)a * BS);
    diag64_store<T>(S, X, WL + (int64_t)(a * BS) * nb + a * BS, nb, Dinv + (int64_t)a * BS * BS,
                    Lf ? Lf + (int64_t)(a * BS) * nb + a * BS : nullptr,
                    If ? If + (int64_t)(a * BS) * nb + a * BS : nullptr);
  } else {
    store64<T, true>(Wab, nb, acc, (T)-1);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_step(T *__restrict__ W, T *__restrict__ WL, int nb,
                                                    int s, T *__restrict__ Dinv, int32_t *flag,
                                                    int64_t colbase, int npairs, T *Winv,
                                                    float *Lf, float *If) {
  potrf_step_body<T>(W, WL, nb, s, Dinv, flag, colbase, blockIdx.x, npairs, Winv, Lf, If);
}

// The steps with the next row tile's panel formed beside them (extra
// workgroups after the pairs and the inverse's).
template <typename T>
__global__ __launch_bounds__(256) void k_potrf_step_row(T *__restrict__ W, T *__restrict__ WL,
                                                        int nb, int s, T *__restrict__ Dinv,
                                                        int32_t *flag, int64_t colbase,
                                                        int npairs, int ninv, T *Winv, float *Lf,
                                                        float *If, RowPanelDev<T> rp) {
  potrf_step_body<T>(W, WL, nb, s, Dinv, flag, colbase, blockIdx.x, npairs, Winv, Lf, If, ninv,
                     &rp);
}

// Inverses of the diagonal tiles k0 .. k0+C-1 (tile c = blockIdx.y or
// blockIdx.z / pairs) by recursive doubling: with the inverses of the
// diagonal blocks of size b known,
//   inv([A 0; B C]) = [inv(A) 0; -inv(C) B inv(A)  inv(C)],
// so each level doubles the block size with two block products.  WL, Dinv:
// the factors and 64-block inverses of all tiles; Winv, Tmp: C tiles.
template <typename T>
__global__ void k_trtri_init(const T *__restrict__ Dinv, T *__restrict__ Winv, int nb, int k0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * nb) return;
  const int c = blockIdx.y, NB = nb / BS;
  const T *D = Dinv + (int64_t)(k0 + c) * NB * BS * BS;
  const int r = (int)(e / nb), q = (int)(e % nb);
  Winv[(int64_t)c * nb * nb + e] =
      (r / BS == q / BS) ? D[(int64_t)(r / BS) * BS * BS + (r % BS) * BS + q % BS] : (T)0;
}

// C = alpha * A * B for b x b blocks (b a multiple of 64), pair p at
// diagonal offset 2 p b.  Output block (blockIdx.y, blockIdx.x) of 64 x 64.
// step 0: Tmp_p = L[(2p+1)b.., 2pb..] * Winv[2pb.., 2pb..]
// step 1: Winv[(2p+1)b.., 2pb..] = -Winv[(2p+1)b.., (2p+1)b..] * Tmp_p
template <typename T>
KRR_DEV void trtri_level_body(const T *__restrict__ WL, T *__restrict__ Winv, T *__restrict__ Tmp,
                              int nb, int b, int step, int64_t p, int rb, int cb) {
  __shared__ T As[BS][BS + 1];
  __shared__ T Bs[BS][BS + 1];
  const int64_t o = 2 * p * b;
  const T *A;
  const T *B;
  T *C;
  int64_t lda, ldb, ldc;
  T alpha;
  if (step == 0) {
    A = WL + (o + b) * nb + o;      lda = nb;
    B = Winv + o * nb + o;          ldb = nb;
    C = Tmp + p * (int64_t)b * b;   ldc = b;
    alpha = (T)1;
  } else {
    A = Winv + (o + b) * nb + o + b; lda = nb;
    B = Tmp + p * (int64_t)b * b;    ldb = b;
    C = Winv + (o + b) * nb + o;     ldc = nb;
    alpha = (T)-1;
  }
  typename M16<T>::v4 acc[4];
  zero4<T>(acc);
  for (int kk = 0; kk < b; kk += BS) {
    load64(As, A + (int64_t)(rb * BS) * lda + kk, lda);
    load64(Bs, B + (int64_t)kk * ldb + cb * BS, ldb);
    __syncthreads();
    mm64<T, false>(As, Bs, acc);
    __syncthreads();
  }
  store64<T, false>(C + (int64_t)(rb * BS) * ldc + cb * BS, ldc, acc, alpha);
}

template <typename T>
__global__ __launch_bounds__(256) void k_trtri_level(const T *__restrict__ WLall,
                                                     T *__restrict__ Winvc, T *__restrict__ Tmpc,
                                                     int nb, int b, int step, int k0, int pairs) {
  const int c = blockIdx.z / pairs;
  const int64_t te = (int64_t)nb * nb;
  trtri_level_body<T>(WLall + (int64_t)(k0 + c) * te, Winvc + (int64_t)c * te,
                      Tmpc + (int64_t)c * (te / 2), nb, b, step, blockIdx.z % pairs, blockIdx.y,
                      blockIdx.x);
}

// Coupling tiles of the paired triangular sweeps, FP32: for the tile pair
// (k, k+1) = (2p, 2p+1) of block lower-triangular L,
//   inv([L_kk 0; L_k+1,k L_k+1,k+1]) = [inv(L_kk) 0; -C_p inv(L_k+1,k+1)],
//   C_p = inv(L_k+1,k+1) L_k+1,k inv(L_kk),
// in two products (step 0: Tmp_p = L_k+1,k inv(L_kk); step 1: C_p =
// inv(L_k+1,k+1) Tmp_p).  Output block (blockIdx.y, blockIdx.x) of 64 x 64 of
// pair blockIdx.z.
__global__ __launch_bounds__(256) void k_sweep_coupling(const float *__restrict__ Lst,
                                                        const float *__restrict__ Linv,
                                                        float *__restrict__ Tmp,
                                                        float *__restrict__ C, int nb, int step) {
  __shared__ float As[BS][BS + 1];
  __shared__ float Bs[BS][BS + 1];
  const int64_t p = blockIdx.z, te = (int64_t)nb * nb, k = 2 * p;
  const int rb = blockIdx.y, cb = blockIdx.x;
  const float *A = step == 0 ? Lst + tri_index(k + 1, k) * te : Linv + (k + 1) * te;
  const float *B = step == 0 ? Linv + k * te : Tmp + p * te;
  float *Out = (step == 0 ? Tmp : C) + p * te;
  typename M16<float>::v4 acc[4];
  zero4<float>(acc);
  for (int kk = 0; kk < nb; kk += BS) {
    load64(As, A + (int64_t)(rb * BS) * nb + kk, nb);
    load64(Bs, B + (int64_t)kk * nb + cb * BS, nb);
    __syncthreads();
    mm64<float, false>(As, Bs, acc);
    __syncthreads();
  }
  store64<float, false>(Out + (int64_t)(rb * BS) * nb + cb * BS, nb, acc, 1.0f);
}

void launch_sweep_coupling(const float *Lst, const float *Linv, const TileLayout &L, float *Tmp,
                           float *C, hipStream_t s) {
  const int npair = L.nt / 2, nbk = L.nb / BS;
  if (npair == 0) return;
  for (int step = 0; step < 2; ++step)
    hipLaunchKernelGGL(k_sweep_coupling, dim3(nbk, nbk, npair), dim3(256), 0, s, Lst, Linv, Tmp, C,
                       L.nb, step);
}

// Coupling of a quad of tiles (k .. k+3, k = 4 q) for sweeps that take four
// tiles a step.  With the pairs P0 = (k, k+1), P1 = (k+2, k+3), M the 2 x 2
// tiles L_{k+2.., k..} between them and inv(P) = [inv(L_a) 0; -C inv(L_b)]
// (C the pair coupling above),
//   inv([P0 0; M P1]) = [inv(P0) 0; -Q inv(P1)],  Q = inv(P1) M inv(P0),
// in two products per tile of Q: stage 0, T = M inv(P0)
//   T00 = L20 inv(L0) - L21 C0,  T01 = L21 inv(L1),
//   T10 = L30 inv(L0) - L31 C0,  T11 = L31 inv(L1);
// stage 1, Q = inv(P1) T
//   Q00 = inv(L2) T00,  Q01 = inv(L2) T01,
//   Q10 = -C1 T00 + inv(L3) T10,  Q11 = -C1 T01 + inv(L3) T11
// (Lij = L_{k+i, k+j}; C0, C1 the couplings of pairs 2q and 2q+1).  Output
// block (blockIdx.y, blockIdx.x) of 64 x 64 of tile blockIdx.z % 4 (00, 01,
// 10, 11) of quad blockIdx.z / 4; each tile a sum of at most two products,
// each in its own FP32 accumulator, added with their signs.
__global__ __launch_bounds__(256) void k_quad_coupling(const float *__restrict__ Lst,
                                                       const float *__restrict__ Linv,
                                                       const float *__restrict__ Cp,
                                                       float *__restrict__ T,
                                                       float *__restrict__ Q, int nb, int stage) {
  __shared__ float As[BS][BS + 1];
  __shared__ float Bs[BS][BS + 1];
  const int64_t te = (int64_t)nb * nb;
  const int o = blockIdx.z % 4;
  const int64_t qd = blockIdx.z / 4, k = 4 * qd;
  const int rb = blockIdx.y, cb = blockIdx.x;
  auto Lt = [&](int i, int j) { return Lst + tri_index(k + i, k + j) * te; };
  auto Li = [&](int i) { return Linv + (k + i) * te; };
  const float *C0 = Cp + (2 * qd) * te, *C1 = Cp + (2 * qd + 1) * te;
  const float *Tq = T + 4 * qd * te;
  const float *A[2] = {nullptr, nullptr}, *B[2] = {nullptr, nullptr};
  float sg[2] = {1.0f, 1.0f};
  if (stage == 0) {
    const int i = 2 + o / 2;  // row tile of M
    if (o % 2 == 0) {
      A[0] = Lt(i, 0), B[0] = Li(0);
      A[1] = Lt(i, 1), B[1] = C0, sg[1] = -1.0f;
    } else {
      A[0] = Lt(i, 1), B[0] = Li(1);
    }
  } else {
    if (o < 2) {
      A[0] = Li(2), B[0] = Tq + o * te;
    } else {
      A[0] = C1, B[0] = Tq + (o - 2) * te, sg[0] = -1.0f;
      A[1] = Li(3), B[1] = Tq + o * te;
    }
  }
  typename M16<float>::v4 acc[2][4];
  zero4<float>(acc[0]);
  zero4<float>(acc[1]);
  for (int t = 0; t < 2; ++t) {
    if (!A[t]) continue;
    for (int kk = 0; kk < nb; kk += BS) {
      load64(As, A[t] + (int64_t)(rb * BS) * nb + kk, nb);
      load64(Bs, B[t] + (int64_t)kk * nb + cb * BS, nb);
      __syncthreads();
      mm64<float, false>(As, Bs, acc[t]);
      __syncthreads();
    }
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[0][ct][e] = sg[0] * acc[0][ct][e] + sg[1] * acc[1][ct][e];
  float *Out = (stage == 0 ? T : Q) + (4 * qd + o) * te;
  store64<float, false>(Out + (int64_t)(rb * BS) * nb + cb * BS, nb, acc[0], 1.0f);
}

void launch_quad_coupling(const float *Lst, const float *Linv, const float *Cpair,
                          const TileLayout &L, float *Tmp, float *Q, hipStream_t s) {
  const int nquad = L.nt / 4, nbk = L.nb / BS;
  if (nquad == 0) return;
  for (int stage = 0; stage < 2; ++stage)
    hipLaunchKernelGGL(k_quad_coupling, dim3(nbk, nbk, 4 * nquad), dim3(256), 0, s, Lst, Linv,
                       Cpair, Tmp, Q, L.nb, stage);
}

// Write L_kk (lower, zero above) into the factor storage and inv(L_kk), FP32.
template <typename T>
__global__ void k_potrf_store(const T *__restrict__ WLall, const T *__restrict__ Winvc,
                              float *__restrict__ Lst, float *__restrict__ Linv, int nb, int k0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)nb * nb) return;
  const int c = blockIdx.y;
  const int64_t k = k0 + c, te = (int64_t)nb * nb;
  const int r = (int)(e / nb), q = (int)(e % nb);
  Lst[(k * (k + 1) / 2 + k) * te + e] = (q <= r) ? (float)WLall[k * te + e] : 0.0f;
  Linv[k * te + e] = (q <= r) ? (float)Winvc[(int64_t)c * te + e] : 0.0f;
}

template <typename T>
static void tile_inverses_t(float *Lst, float *Linv, int k_lo, int k_hi, const TileLayout &L,
                            FactorWork &w, hipStream_t s) {
  const int nb = L.nb;
  const unsigned eb = (unsigned)(((int64_t)nb * nb + 255) / 256);
  for (int k0 = k_lo; k0 < k_hi; k0 += w.inv_chunk) {
    const int C = std::min(w.inv_chunk, k_hi - k0);
    hipLaunchKernelGGL(k_trtri_init<T>, dim3(eb, C), dim3(256), 0, s, (const T *)w.Dinv64,
                       (T *)w.Winv64, nb, k0);
    for (int b = BS; b < nb; b *= 2) {
      const unsigned nbk = (unsigned)(b / BS);
      const int pairs = nb / (2 * b);
      for (int step = 0; step < 2; ++step)
        hipLaunchKernelGGL(k_trtri_level<T>, dim3(nbk, nbk, pairs * C), dim3(256), 0, s,
                           (const T *)w.WL64, (T *)w.Winv64, (T *)w.Tmp64, nb, b, step, k0,
                           pairs);
    }
    hipLaunchKernelGGL(k_potrf_store<T>, dim3(eb, C), dim3(256), 0, s, (const T *)w.WL64,
                       (const T *)w.Winv64, Lst, Linv, nb, k0);
  }
}

void launch_tile_inverses(float *Lst, float *Linv, int k_lo, int k_hi, const TileLayout &L,
                          bool fp64, FactorWork &w, hipStream_t s) {
  if (fp64)
    tile_inverses_t<double>(Lst, Linv, k_lo, k_hi, L, w, s);
  else
    tile_inverses_t<float>(Lst, Linv, k_lo, k_hi, L, w, s);
}

// Load the diagonal tile with its last updates folded in:
//   W = A_kk - sum_q P_q P_q^T   (lower 64 x 64 blocks; the upper ones are never read)
// where P_q is tile k of panel buffer q (the panels whose update of this tile
// was left to the factorization), as an FP32 MFMA product with FP32
// accumulation -- the same arithmetic as the trailing update of a diagonal
// tile -- and the difference formed in T.
typedef GemmShape<64, 64, 2, 2> DiagUpdShape;

// With If (the tile's FP32 inverse) the workgroup of block (bi, bj), bi > bj,
// also zeroes block (bj, bi) above the diagonal of Akk and of If: the FP32
// factor and inverse are then written into those tiles block by block during
// the factorization, and their upper blocks stay zero.
template <typename T>
KRR_DEV void potrf_load_body(float *__restrict__ Akk, T *__restrict__ W, int nb,
                             const DiagUpdate &du, int bid, float *__restrict__ If = nullptr) {
  typedef DiagUpdShape S;
  __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];
  int bi, bj;
  tri_decode(bid, bi, bj);
  OpF32::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  for (int q = 0; q < du.npan; ++q)
    gemm_nt_core<OpF32, S>(OpF32{}, (const uint8_t *)(du.P[q] + (int64_t)bi * 64 * nb),
                           (int64_t)nb * 4, 64, (const uint8_t *)(du.P[q] + (int64_t)bj * 64 * nb),
                           (int64_t)nb * 4, 64, (int64_t)nb * 4, acc, lds);
  if (bid == 0 && threadIdx.x < du.npan && du.pmap)
    du.pmap[du.pmap_at[threadIdx.x]] = (uint8_t)KRR_PREC_FP32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // every entry of the block loaded (upper ones too: they are in the tile),
  // all loads in flight before the first use: a load under the c <= r
  // condition would take a round trip of its own
  float av[S::WTM][S::WTN][16];
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = bi * 64 + S::row(wave, tm, e, lane), c = bj * 64 + S::col(wave, tn, lane);
        av[tm][tn][e] = Akk[(int64_t)r * nb + c];
      }
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e) asm volatile("" : "+v"(av[tm][tn][e]));
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int r = bi * 64 + S::row(wave, tm, e, lane), c = bj * 64 + S::col(wave, tn, lane);
        const int64_t o = (int64_t)r * nb + c;
        W[o] = (c <= r) ? (T)av[tm][tn][e] - (T)acc[tm][tn][e] : (T)0;
      }
  if (If && bi > bj) {
    __syncthreads();  // every read of this workgroup's block is done (it is not the zeroed one)
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int64_t o = (int64_t)(bj * 64 + e / 64) * nb + bi * 64 + e % 64;
      Akk[o] = 0.0f;
      If[o] = 0.0f;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_load(float *__restrict__ Akk, T *__restrict__ W,
                                                    int nb, DiagUpdate du, float *If) {
  potrf_load_body<T>(Akk, W, nb, du, blockIdx.x, If);
}

// The same load split over K, for one instance, in two launches.  First,
// workgroup (blk, c) forms chunk c of the product (kc values of k of one
// panel) for 64 x 64 block blk into a slot of its own; then one workgroup
// per block adds the slots in chunk order and forms W = A - sum (the same
// FP32 products, summed per chunk), and the one of block (0, 0) factors and
// inverts it at once (the tile's first 64-column step, otherwise a launch of
// its own).  The launch boundary orders the slots: no workgroup waits for
// another and no device-wide fence is needed.
__global__ __launch_bounds__(256) void k_potrf_load_part(int nb, DiagUpdate du, int kc,
                                                         float *__restrict__ part) {
  typedef DiagUpdShape S;
  __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];
  const int NB = nb / BS, nblk = NB * (NB + 1) / 2, cpp = nb / kc;
  const int blk = (int)(blockIdx.x % nblk), c = (int)(blockIdx.x / nblk);
  int bi, bj;
  tri_decode(blk, bi, bj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  OpF32::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  const float *P = du.P[c / cpp] + (c % cpp) * kc;
  gemm_nt_core<OpF32, S>(OpF32{}, (const uint8_t *)(P + (int64_t)bi * 64 * nb), (int64_t)nb * 4,
                         64, (const uint8_t *)(P + (int64_t)bj * 64 * nb), (int64_t)nb * 4, 64,
                         (int64_t)kc * 4, acc, lds);
  float *slot = part + ((int64_t)c * nblk + blk) * (BS * BS);
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e)
        slot[S::row(wave, tm, e, lane) * BS + S::col(wave, tn, lane)] = acc[tm][tn][e];
}

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_load_sum(float *__restrict__ Akk,
                                                        T *__restrict__ W, T *__restrict__ WL,
                                                        int nb, DiagUpdate du, int nch,
                                                        const float *__restrict__ part,
                                                        T *__restrict__ Dinv, int32_t *flag,
                                                        int64_t colbase, float *Lf, float *If) {
  __shared__ T Sb[BS][BS + 1];  // block (0, 0), overwritten by its factor
  __shared__ T Xb[BS][BS + 1];  // and its inverse
  const int NB = nb / BS, nblk = NB * (NB + 1) / 2;
  const int blk = blockIdx.x;
  int bi, bj;
  tri_decode(blk, bi, bj);
  if (blk == 0 && threadIdx.x < du.npan && du.pmap)
    du.pmap[du.pmap_at[threadIdx.x]] = (uint8_t)KRR_PREC_FP32;
  // four runs of four entries a thread; every slot and A load in flight at
  // once (chunks past nch read as zeros, which leave the ordered sum as it is)
  const float *slots = part + (int64_t)blk * (BS * BS);
  const int64_t stride = (int64_t)nblk * (BS * BS);
  float4 v[4][KRR_MAX_GROUP], a[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int e = 4 * (threadIdx.x + 256 * g), r = e / BS, cc = e % BS;
    a[g] = *(const float4 *)(Akk + (int64_t)(bi * BS + r) * nb + bj * BS + cc);
#pragma unroll
    for (int q = 0; q < KRR_MAX_GROUP; ++q)
      v[g][q] = q < nch ? *(const float4 *)(slots + q * stride + e)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int e = 4 * (threadIdx.x + 256 * g), r = e / BS, cc = e % BS;
    float4 sum = v[g][0];
#pragma unroll
    for (int q = 1; q < KRR_MAX_GROUP; ++q) {
      sum.x += v[g][q].x;
      sum.y += v[g][q].y;
      sum.z += v[g][q].z;
      sum.w += v[g][q].w;
    }
    const float av[4] = {a[g].x, a[g].y, a[g].z, a[g].w};
    const float sv[4] = {sum.x, sum.y, sum.z, sum.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T val = (bj * BS + cc + j <= bi * BS + r) ? (T)av[j] - (T)sv[j] : (T)0;
      W[(int64_t)(bi * BS + r) * nb + bj * BS + cc + j] = val;
      if (blk == 0) Sb[r][cc + j] = val;
    }
  }
  if (If && bi > bj) {  // the upper block, for the factor and inverse written in the steps
    __syncthreads();    // (not read here: only lower entries are)
    for (int e = threadIdx.x; e < BS * BS; e += 256) {
      const int64_t o = (int64_t)(bj * BS + e / BS) * nb + bi * BS + e % BS;
      Akk[o] = 0.0f;
      If[o] = 0.0f;
    }
  }
  if (blk == 0) {
    __syncthreads();
    diag64_body<T>(Sb, Xb, flag, colbase);
    diag64_store<T>(Sb, Xb, WL, nb, Dinv, Lf, If);
  }
}

// The FP64 (or FP32) inverse of tile k while it is formed in the steps: one of
// two slots of the chunk buffer, so that the next tile's steps may run while
// the last block row of this one is still being formed.
template <typename T>
static T *inv_slot(FactorWork &w, int k, int64_t te) {
  return (T *)w.Winv64 + (int64_t)(k % 2) * te;
}

template <typename T>
static void potrf_tile_t(float *Akk, int k, const TileLayout &L, FactorWork &w,
                         const DiagUpdate &du, float *Linv_k, hipStream_t s,
                         const RowPanel &row) {
  const int nb = L.nb, NB = nb / BS;
  const int64_t te = (int64_t)nb * nb;
  T *W = (T *)w.W64, *WL = (T *)w.WL64 + k * te, *Dinv = (T *)w.Dinv64 + (int64_t)k * NB * BS * BS;
  T *Winv = Linv_k ? inv_slot<T>(w, k, te) : nullptr;
  float *Lf = Linv_k ? Akk : nullptr;
  const int64_t colbase = (int64_t)k * nb;
  const char *e = getenv("KRR_LOAD_SPLIT");
  if (w.lpart && du.npan > 0 && !(e && atoi(e) == 0)) {
    // K chunks: a whole panel each from four panels up, else halves or quarters
    const int cpp = du.npan >= 4 ? 1 : (du.npan >= 2 ? 2 : 4), nch = du.npan * cpp;
    const int nblk = NB * (NB + 1) / 2;
    hipLaunchKernelGGL(k_potrf_load_part, dim3(nblk * nch), dim3(256), 0, s, nb, du, nb / cpp,
                       w.lpart);
    hipLaunchKernelGGL(k_potrf_load_sum<T>, dim3(nblk), dim3(256), 0, s, Akk, W, WL, nb, du, nch,
                       w.lpart, Dinv, w.flag, colbase, Lf, Linv_k);
  } else {
    hipLaunchKernelGGL(k_potrf_load<T>, dim3(NB * (NB + 1) / 2), dim3(256), 0, s, Akk, W, nb, du,
                       Linv_k);
    hipLaunchKernelGGL(k_potrf_diag64<T>, dim3(1), dim3(256), 0, s, W, WL, nb, Dinv, w.flag,
                       colbase, Lf, Linv_k);
  }
  const bool with_row = row.A && w.WX64;
  RowPanelDev<T> rp{row.A, (T *)w.WX64, row.P32, row.pnorm_part, row.pmax_part, row.parts, 0};
  if (with_row && row.wait) (void)hipStreamWaitEvent(s, row.wait, 0);  // A_k+1,k complete
  for (int st = 0; st + 1 < NB; ++st) {
    const int rest = NB - 1 - st, npairs = rest * (rest + 1) / 2;
    // the inverse: row st finalized, the later rows' sums advanced by row st - 1
    const int ninv = Winv ? st + (NB - 1 - st) * st : 0;
    if (with_row)
      hipLaunchKernelGGL(k_potrf_step_row<T>, dim3(npairs + ninv + NB * rest), dim3(256), 0, s, W,
                         WL, nb, st, Dinv, w.flag, colbase, npairs, ninv, Winv, Lf, Linv_k, rp);
    else
      hipLaunchKernelGGL(k_potrf_step<T>, dim3(npairs + ninv), dim3(256), 0, s, W, WL, nb, st,
                         Dinv, w.flag, colbase, npairs, Winv, Lf, Linv_k);
  }
  if (with_row) {  // the panel's last block column
    rp.final_launch = 1;
    hipLaunchKernelGGL(k_potrf_step_row<T>, dim3(NB), dim3(256), 0, s, W, WL, nb, NB - 1, Dinv,
                       w.flag, colbase, 0, 0, Winv, Lf, Linv_k, rp);
  }
}

void launch_potrf_tile(float *Akk, int k, const TileLayout &L, bool fp64, FactorWork &w,
                       const DiagUpdate &du, float *Linv_k, hipStream_t s, const RowPanel &row) {
  if (fp64)
    potrf_tile_t<double>(Akk, k, L, w, du, Linv_k, s, row);
  else
    potrf_tile_t<float>(Akk, k, L, w, du, Linv_k, s, row);
}

void launch_tile_inverse_last_row(float *Linv_k, int k, const TileLayout &L, bool fp64,
                                  FactorWork &w, hipStream_t s) {
  const int nb = L.nb, NB = nb / BS;
  const int64_t te = (int64_t)nb * nb;
  if (NB < 2) return;
  if (fp64)
    hipLaunchKernelGGL(k_potrf_step<double>, dim3(NB - 1), dim3(256), 0, s, (double *)w.W64,
                       (double *)w.WL64 + k * te, nb, NB - 1,
                       (double *)w.Dinv64 + (int64_t)k * NB * BS * BS, w.flag, (int64_t)k * nb, 0,
                       inv_slot<double>(w, k, te), (float *)nullptr, Linv_k);
  else
    hipLaunchKernelGGL(k_potrf_step<float>, dim3(NB - 1), dim3(256), 0, s, (float *)w.W64,
                       (float *)w.WL64 + k * te, nb, NB - 1,
                       (float *)w.Dinv64 + (int64_t)k * NB * BS * BS, w.flag, (int64_t)k * nb, 0,
                       inv_slot<float>(w, k, te), (float *)nullptr, Linv_k);
}

// ---------------------------------------------------------------------------
// Panel TRSM: P_i = A_ik inv(L_kk)^T, i.e. P_i L_kk^T = A_ik, by block forward
// substitution with the diagonal tile's factor and its 64-block inverses:
//   P[:, s] = (A[:, s] - sum_{t<s} P[:, t] L_st^T) inv(L_ss)^T,  s = 0 .. nb/64-1.
// Rows are independent: one workgroup per 16 rows of one tile i = k+1+t
// (t_lo <= t), keeping its rows of P in LDS in T (the diagonal factor's
// precision); wave w owns columns 16w .. 16w+15 of each 64-column block.
// The panel buffer gets P in FP32, and each workgroup leaves the FP64 sum of
// squares and the max |entry| of its rows (for the operand norms and scales).
// It needs no inverse of the whole tile, so no tile inverse lies on the
// factorization's critical path.
constexpr int TRSM_ROWS = 16;

template <typename T>
KRR_DEV void trsm_panel_body(const float *__restrict__ Astore, const T *__restrict__ WLk,
                             const T *__restrict__ Dinvk, int k, int t_lo, int nb, int parts,
                             float *__restrict__ P32, double *__restrict__ pnorm_part,
                             float *__restrict__ pmax_part, int bid) {
  typedef typename M16<T>::v4 v4;
  __shared__ T Pr[TRSM_ROWS][512 + 1];
  __shared__ T Tb[TRSM_ROWS][BS + 1];
  __shared__ double shd[4];
  __shared__ float shf[4];
  const int RS = nb / TRSM_ROWS;
  const int64_t t = t_lo + bid / RS;
  const int r0 = (bid % RS) * TRSM_ROWS;
  const int64_t i = k + 1 + t, te = (int64_t)nb * nb;
  const float *A = Astore + (i * (i + 1) / 2 + k) * te + (int64_t)r0 * nb;
  float *Pout = P32 + t * te + (int64_t)r0 * nb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
  double ss = 0.0;
  float mx = 0.0f;
  // Sixteen MFMAs over 64 values of k, A(li, k) = a[4 u + lg] from LDS and
  // B = b[u]: all sixteen LDS reads issued first (each into a register of its
  // own), the MFMAs alternating between two accumulators (even and odd u,
  // added by the caller) so that no MFMA waits for the one before it.
  auto mma_chunk = [&](const T *a, const T (&b)[16], v4 &e, v4 &o) {
    T pa[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) pa[u] = a[4 * u];
#pragma unroll
    for (int u = 0; u < 16; u += 2) {
      e = M16<T>::mma(pa[u], b[u], e);
      o = M16<T>::mma(pa[u + 1], b[u + 1], o);
    }
    __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
  };
  for (int s = 0; s < nb / BS; ++s) {
    const int c0 = BS * s + 16 * wave;  // this wave's 16 output columns
    // this step's A entries and inv(L_ss) row, loaded before the sum so that
    // their latency overlaps it
    float av[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) av[r] = A[(int64_t)M16<T>::row(r, lane) * nb + c0 + li];
    const T *Drow = Dinvk + (int64_t)s * BS * BS + (16 * wave + li) * BS;
    T dv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) dv[u] = Drow[4 * u + lg];
    // B(kk, c) = L[c0 + c][kk] over kk < 64 s, 64 columns of k per chunk;
    // the loads of chunk c+1 are issued before the MFMAs of chunk c
    const T *Lrow = WLk + (int64_t)(c0 + li) * nb;
    v4 acc = {0, 0, 0, 0}, acc_o = {0, 0, 0, 0};
    const int nch = s;
    if (nch > 0) {
      T b0[16], b1[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) b0[u] = Lrow[4 * u + lg];
      for (int ch = 0; ch < nch; ch += 2) {
        const int k0 = BS * ch;
        if (ch + 1 < nch) {
#pragma unroll
          for (int u = 0; u < 16; ++u) b1[u] = Lrow[k0 + BS + 4 * u + lg];
        }
        mma_chunk(Pr[li] + k0 + lg, b0, acc, acc_o);
        if (ch + 1 < nch) {
          if (ch + 2 < nch) {
#pragma unroll
            for (int u = 0; u < 16; ++u) b0[u] = Lrow[k0 + 2 * BS + 4 * u + lg];
          }
          mma_chunk(Pr[li] + k0 + BS + lg, b1, acc, acc_o);
        }
      }
    }
    acc += acc_o;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = M16<T>::row(r, lane);
      Tb[row][16 * wave + li] = (T)av[r] - acc[r];
    }
    __syncthreads();
    // P[:, c0 ..] = Tb inv(L_ss)^T: B(j, c) = inv(L_ss)[16 w + c][j]
    v4 acc2 = {0, 0, 0, 0}, acc2_o = {0, 0, 0, 0};
    mma_chunk(Tb[li] + lg, dv, acc2, acc2_o);
    acc2 += acc2_o;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = M16<T>::row(r, lane);
      const float f = (float)acc2[r];
      Pr[row][c0 + li] = acc2[r];
      Pout[(int64_t)row * nb + c0 + li] = f;
      ss += (double)f * (double)f;
      mx = fmaxf(mx, fabsf(f));
    }
    __syncthreads();
  }
  ss = block_sum<4>(ss, shd);
  mx = block_max<4>(mx, shf);
  if (threadIdx.x == 0) {
    pnorm_part[t * parts + bid % RS] = ss;
    pmax_part[t * parts + bid % RS] = mx;
  }
  // a tile has `parts` slots; the ones past RS stay empty here
  if (bid % RS == 0 && threadIdx.x >= RS && threadIdx.x < parts) {
    pnorm_part[t * parts + threadIdx.x] = 0.0;
    pmax_part[t * parts + threadIdx.x] = 0.0f;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsm_panel(const float *__restrict__ Astore,
                                                    const T *__restrict__ WLk,
                                                    const T *__restrict__ Dinvk, int k, int t_lo,
                                                    int nb, int parts, float *__restrict__ P32,
                                                    double *__restrict__ pnorm_part,
                                                    float *__restrict__ pmax_part) {
  trsm_panel_body<T>(Astore, WLk, Dinvk, k, t_lo, nb, parts, P32, pnorm_part, pmax_part,
                     blockIdx.x);
}

// Partial-norm slots per tile: the substitution TRSM fills nb/16 of them, the
// product form one per 64 x 64 block.
int trsm_parts(int nb) { return std::max((nb / 64) * (nb / 64), nb / TRSM_ROWS); }

template <typename T>
static void trsm_subst_t(const float *Astore, int k, const TileLayout &L, FactorWork &w,
                         const PanelBuf &pb, int t_lo, int t_hi, hipStream_t s) {
  const int nb = L.nb, RS = nb / TRSM_ROWS, NB = nb / BS;
  const int64_t te = (int64_t)nb * nb;
  hipLaunchKernelGGL(k_trsm_panel<T>, dim3((unsigned)((t_hi - t_lo) * RS)), dim3(256), 0, s, Astore,
                     (const T *)w.WL64 + k * te, (const T *)w.Dinv64 + (int64_t)k * NB * BS * BS,
                     k, t_lo, nb, trsm_parts(nb), pb.P32, w.pnorm_part, w.pmax_part);
}

void launch_trsm_subst(const float *Astore, int k, const TileLayout &L, bool fp64, FactorWork &w,
                       const PanelBuf &pb, int t_lo, int t_hi, hipStream_t s) {
  t_hi = std::min(t_hi, L.nt - 1 - k);
  if (t_hi <= t_lo) return;
  if (fp64)
    trsm_subst_t<double>(Astore, k, L, w, pb, t_lo, t_hi, s);
  else
    trsm_subst_t<float>(Astore, k, L, w, pb, t_lo, t_hi, s);
}

// Panel TRSM as an FP32 MFMA product with the tile inverse:
// P_i = A_ik inv(L_kk)^T for the tiles i = k+1+t, t >= t_lo, 64 x 64 blocks,
// each leaving its FP64 sum of squares and max |entry|.
typedef GemmShape<64, 64, 2, 2> TrsmShape;

KRR_DEV void trsm_gemm_body(const float *__restrict__ Astore, const float *__restrict__ Linv,
                           int k, int t_lo, int nb, int parts, float *__restrict__ P32,
                           double *__restrict__ pnorm_part, float *__restrict__ pmax_part,
                           int64_t bid) {
  typedef TrsmShape S;
  constexpr int B = S::kBM;
  __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS_BYTES];
  __shared__ double shd[4];
  __shared__ float shf[4];
  const int SB = nb / B, nsub = SB * SB;
  const int sub = (int)(bid % nsub);
  const int64_t t = t_lo + bid / nsub;
  const int64_t i = k + 1 + t;
  const int si = sub / SB, sj = sub % SB;
  const int64_t te = (int64_t)nb * nb;
  const float *Ablk = Astore + (i * (i + 1) / 2 + k) * te + (int64_t)si * B * nb;
  const float *Bblk = Linv + (int64_t)sj * B * nb;
  const int64_t kbytes = (int64_t)min(nb, (sj + 1) * B) * 4;  // inv(L) is lower triangular
  OpF32::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  gemm_nt_core<OpF32, S>(OpF32{}, (const uint8_t *)Ablk, (int64_t)nb * 4, B, (const uint8_t *)Bblk,
                         (int64_t)nb * 4, B, kbytes, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float *out = P32 + t * te + (int64_t)si * B * nb + sj * B;
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
    pnorm_part[t * parts + sub] = ss;
    pmax_part[t * parts + sub] = mx;
  }
  if (sub == 0 && threadIdx.x >= nsub && threadIdx.x < parts) {
    pnorm_part[t * parts + threadIdx.x] = 0.0;
    pmax_part[t * parts + threadIdx.x] = 0.0f;
  }
}

__global__ __launch_bounds__(256) void k_trsm_gemm(const float *__restrict__ Astore,
                                                   const float *__restrict__ Linv, int k, int t_lo,
                                                   int nb, int parts, float *__restrict__ P32,
                                                   double *__restrict__ pnorm_part,
                                                   float *__restrict__ pmax_part) {
  trsm_gemm_body(Astore, Linv, k, t_lo, nb, parts, P32, pnorm_part, pmax_part,
                 xcd_remap(blockIdx.x, gridDim.x));
}

void launch_trsm_gemm(const float *Astore, const float *Linv_k, int k, const TileLayout &L,
                      FactorWork &w, const PanelBuf &pb, int t_lo, int t_hi, hipStream_t s) {
  t_hi = std::min(t_hi, L.nt - 1 - k);
  if (t_hi <= t_lo) return;
  const int SB = L.nb / TrsmShape::kBM;
  hipLaunchKernelGGL(k_trsm_gemm, dim3((unsigned)((t_hi - t_lo) * SB * SB)), dim3(256), 0, s,
                     Astore, Linv_k, k, t_lo, L.nb, trsm_parts(L.nb), pb.P32, w.pnorm_part,
                     w.pmax_part);
}

// Panel conversion: reduce each tile's partial norms (fixed order), pick the
// FP8 power-of-two scale, copy the FP32 L_ik into the factor storage and
// write the FP16 copy (unscaled) and the scaled FP8 E4M3 copy.
// elements per workgroup (nb^2 is a multiple of both): one instance's panels
// run beside other work and want many small workgroups; the lockstep batch
// has many instances per launch and wants fewer, longer ones
constexpr int CONV_CHUNK = 4096, CONV_CHUNK_B = 16384;

// The precision the rule chooses for an operand-norm product, before the
// precisions the attempt allows and the panel caps are applied.
KRR_DEV int rule_prec(const UpdatePolicy &pol, double prod) {
  if (pol.allow8 && 0.0625 * prod <= pol.thr) return KRR_PREC_FP8;
  if (pol.allow16 && 0.00048828125 * prod <= pol.thr) return KRR_PREC_FP16;
  return KRR_PREC_FP32;
}

// The precision an update reads its operands in: the choice c capped by the
// panel's promotion level, FP16 only where FP16 operands are reachable.
KRR_DEV int effective_prec(const UpdatePolicy &pol, int k, int c) {
  if (pol.pcap && c > (int)pol.pcap[k]) c = pol.pcap[k];
  if (c == KRR_PREC_FP8 && !pol.allow8) c = KRR_PREC_FP16;
  if (c == KRR_PREC_FP16 && !pol.have16) c = KRR_PREC_FP32;
  return c;
}

// Which copies of panel k's tile with norm pn some update will read (its
// partners' norms lie in [mn, mx]): the effective precisions of the choices
// between those of pn mx and pn mn under the operand rule, the fixed
// precision under FIXED, every allowed one under the map or the tile rules.
KRR_DEV void copies_needed(const UpdatePolicy &pol, int k, float pn, float mn, float mx, int &n16,
                           int &n8) {
  int lo = KRR_PREC_FP32, hi = KRR_PREC_FP32;
  if (pol.mode == KRR_POLICY_FIXED_MAP ||
      (pol.mode == KRR_POLICY_ADAPTIVE && pol.rule != KRR_RULE_OPERAND && k >= pol.high_panels)) {
    hi = KRR_PREC_FP8;
  } else if (k >= pol.high_panels && pol.mode == KRR_POLICY_FIXED) {
    lo = hi = pol.fixed_prec;
  } else if (k >= pol.high_panels && pol.mode == KRR_POLICY_ADAPTIVE) {
    lo = rule_prec(pol, (double)pn * (double)mx);
    hi = rule_prec(pol, (double)pn * (double)mn);
  }
  n16 = n8 = 0;
  for (int c = lo; c <= hi; ++c) {
    const int e = effective_prec(pol, k, c);
    n16 |= e == KRR_PREC_FP16;
    n8 |= e == KRR_PREC_FP8;
  }
}

// Panel k's tile norms (each tile's partial sums added in a fixed order, as
// FP32) and, at pnorm[mm_at] and pnorm[mm_at + 1], their smallest and largest.
__global__ __launch_bounds__(256) void k_panel_norms(const double *__restrict__ pnorm_part,
                                                     int parts, int tiles,
                                                     float *__restrict__ pnorm, int mm_at) {
  __shared__ float smn[256], smx[256];
  float mn = INFINITY, mx = 0.0f;
  for (int t = threadIdx.x; t < tiles; t += 256) {
    double ss = 0.0;
    for (int q = 0; q < parts; ++q) ss += pnorm_part[(int64_t)t * parts + q];
    const float v = (float)sqrt(ss);
    pnorm[t] = v;
    mn = fminf(mn, v);
    mx = fmaxf(mx, v);
  }
  smn[threadIdx.x] = mn;
  smx[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smn[threadIdx.x] = fminf(smn[threadIdx.x], smn[threadIdx.x + w]);
      smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pnorm[mm_at] = smn[0];
    pnorm[mm_at + 1] = smx[0];
  }
}

// select: the tile norms and their extremes are in pnorm already (from
// k_panel_norms) and only the copies pol lets some update read are written;
// otherwise the norms are formed here and need16 / need8 decide.
KRR_DEV void convert_panel_body(const float *__restrict__ P32, float *__restrict__ Astore,
                                _Float16 *__restrict__ P16, uint8_t *__restrict__ P8,
                                const double *__restrict__ pnorm_part,
                                const float *__restrict__ pmax_part, int parts,
                                float *__restrict__ pnorm, int *__restrict__ pexp8, int k, int nb,
                                int chunks, int need16, int need8, int scale8, int64_t bid,
                                int select = 0, const UpdatePolicy *pol = nullptr,
                                int mm_at = 0) {
  const int64_t t = bid / chunks;
  const int ch = (int)(bid % chunks);
  const int64_t i = k + 1 + t;
  if (select) copies_needed(*pol, k, pnorm[t], pnorm[mm_at], pnorm[mm_at + 1], need16, need8);
  // the tile's largest magnitude from its partial maxima, one per thread
  // (a max is exact in any order)
  __shared__ float smx[256];
  {
    float m = 0.0f;
    for (int q = threadIdx.x; q < parts; q += 256) m = fmaxf(m, pmax_part[t * parts + q]);
    smx[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + w]);
      __syncthreads();
    }
  }
  const float mx = smx[0];
  const float s8 = scale8 ? pow2_scale(mx, 448.0f) : 1.0f;
  const int64_t te = (int64_t)nb * nb;
  const float *src = P32 + t * te;
  float *dstL = Astore + (i * (i + 1) / 2 + k) * te;
  const int64_t csz = te / chunks, e0 = (int64_t)ch * csz;
  for (int64_t e = e0 + threadIdx.x * 4; e < e0 + csz; e += 256 * 4) {
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
    if (!select) {
      double ss = 0.0;  // the tile norm, partial sums added in a fixed order
      for (int q = 0; q < parts; ++q) ss += pnorm_part[t * parts + q];
      pnorm[t] = (float)sqrt(ss);
    }
    pexp8[t] = ilogbf(s8);  // s8 = 2^pexp8
  }
}

__global__ __launch_bounds__(256) void k_convert_panel(
    const float *__restrict__ P32, float *__restrict__ Astore, _Float16 *__restrict__ P16,
    uint8_t *__restrict__ P8, const double *__restrict__ pnorm_part,
    const float *__restrict__ pmax_part, int parts, float *__restrict__ pnorm,
    int *__restrict__ pexp8, int k, int nb, int chunks, int need16, int need8, int scale8,
    int select, UpdatePolicy pol, int mm_at) {
  convert_panel_body(P32, Astore, P16, P8, pnorm_part, pmax_part, parts, pnorm, pexp8, k, nb,
                     chunks, need16, need8, scale8, blockIdx.x, select, &pol, mm_at);
}

void launch_convert_panel(float *Astore, int k, const TileLayout &L, FactorWork &w, bool scale8,
                          const PanelBuf &pb, bool need16, bool need8, const UpdatePolicy *pol,
                          hipStream_t s) {
  const int64_t tiles = L.nt - 1 - k;
  if (tiles <= 0) return;
  const int chunks = (int)((int64_t)L.nb * L.nb / CONV_CHUNK);
  const int mm_at = std::max(L.nt - 1, 1);  // the norms' extremes after the largest panel
  const int parts = trsm_parts(L.nb);
  if (pol)
    hipLaunchKernelGGL(k_panel_norms, dim3(1), dim3(256), 0, s, w.pnorm_part, parts, (int)tiles,
                       pb.pnorm, mm_at);
  hipLaunchKernelGGL(k_convert_panel, dim3((unsigned)(tiles * chunks)), dim3(256), 0, s, pb.P32,
                     Astore, pb.P16, pb.P8, w.pnorm_part, w.pmax_part, parts, pb.pnorm,
                     pb.pexp8, k, L.nb, chunks, need16 ? 1 : 0, need8 ? 1 : 0, scale8 ? 1 : 0,
                     pol ? 1 : 0, pol ? *pol : UpdatePolicy{}, mm_at);
}

// Trailing update by a group of consecutive panels k0 .. k0+npan-1:
//   A_ij -= sum_k L_ik L_jk^T   for the tiles (i, j), jlo <= j <= jhi, j <= i < NT,
// one 256 x 256 (off-diagonal) or 128 x 128 (diagonal tiles, short column
// ranges) block per workgroup, FP32 accumulation over all panels of the
// group, subtracted from C once per element (each element belongs to one
// workgroup of the launch, and no other launch touches the tile meanwhile).  The operand
// precision is chosen per (tile, panel), uniform across the workgroup:
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

// Trailing update of one group of panels: sub-block (si, sj) of tile (i, j)
// (256 x 256 off the diagonal, 128 x 128 on it) gets
// A_ij -= sum_q L_i,k0+q L_j,k0+q^T.  Each panel's operands
// take the precision chosen for this update; the panels of one precision
// form one streamed K range (one segment per panel), so a sub-block runs at
// most three products (FP32, FP16, FP8 operands) into one FP32 accumulator.
typedef StreamShape<256, 256, 2, 4, 4> UpdStream;   // off-diagonal tiles
typedef StreamShape<128, 128, 2, 2, 4> UpdDiagStream;  // few off-diagonal tiles
// Diagonal tiles: always FP32 and with up to a whole group of
// panels (K = 8 nb), so each block's serial K loop is long; 64 x 64 blocks
// cut it four times over and give four times the workgroups.
typedef StreamShape<64, 64, 2, 2, 4> UpdDiag64;

// Segment table in LDS: per precision, the row-0 addresses of the A and B
// operand blocks of each selected panel (and the FP8 scale codes).
struct SegTable {
  uint64_t a[3][KRR_MAX_GROUP];
  uint64_t b[3][KRR_MAX_GROUP];
  int sa[KRR_MAX_GROUP], sb[KRR_MAX_GROUP];
  int cnt[3];
};

typedef const __attribute__((address_space(3))) SegTable *LdsSegTable;
typedef const __attribute__((address_space(3))) uint64_t *LdsU64;

template <class Op>
struct SegSrc {
  LdsSegTable t;  // LDS address space: plain LDS reads, no flat accesses
  int p, sh;      // precision index, log2(slabs per panel)
  KRR_DEV uint64_t seg_base(LdsU64 v, int64_t s) const {
    const uint64_t x = v[s >> sh];
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32 | lo) + (uint64_t)((s & ((1 << sh) - 1)) << 6);
  }
  KRR_DEV const uint8_t *ptr(bool side_a, int64_t s) const {
    return (const uint8_t *)seg_base(side_a ? t->a[p] : t->b[p], s);
  }
  KRR_DEV Op op(int64_t s) const {
    if constexpr (std::is_same<Op, OpF8>::value) {
      OpF8 o;
      o.sa = __builtin_amdgcn_readfirstlane(t->sa[s >> sh]);
      o.sb = __builtin_amdgcn_readfirstlane(t->sb[s >> sh]);
      return o;
    } else {
      return Op{};
    }
  }
};

// DIAG: the diagonal tiles (j, j), jlo <= j <= jhi -- FP32 operands, the
// longest work per output, so they run in smaller blocks of their own launch
// (lower sub-blocks only).  Otherwise the off-diagonal tiles, remapped so that
// the sub-blocks of one tile share an XCD.
template <class S, bool DIAG>
KRR_DEV void update_body(float *__restrict__ Astore, const PanelSet &ps, int k0, int npan, int jlo,
                         int jhi, int NT, int nb, int SB, const UpdatePolicy &pol,
                         uint8_t *__restrict__ pmap, int64_t ntiles_all, int64_t blk,
                         int64_t nblk) {
  constexpr int BM = S::kBM;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  __shared__ SegTable tab;
  int64_t i, j;
  int si, sj;
  if constexpr (DIAG) {
    const int nsd = SB * (SB + 1) / 2;
    i = j = jlo + blk / nsd;
    tri_decode(blk % nsd, si, sj);
  } else {
    const int nsub = SB * SB;
    const int64_t bid = xcd_remap(blk, nblk);
    const int sub = (int)(bid % nsub);
    int64_t tt = bid / nsub;
    si = sub / SB;
    sj = sub % SB;
    if (jhi == NT - 1) {  // strict lower triangle of the tiles right of column jlo
      int ta, tb;
      tri_decode(tt, ta, tb);
      i = jlo + ta + 1;
      j = jlo + tb;
    } else {  // a few columns: walk them
      j = jlo;
      while (tt >= NT - 1 - j) {
        tt -= NT - 1 - j;
        ++j;
      }
      i = j + 1 + tt;
    }
  }
  const int64_t te = (int64_t)nb * nb;
  const bool first_sub = (si == 0 && sj == 0);

  // Thread q < npan picks the operand precision of panel q (all panels'
  // loads in flight together); thread 0 then lists the panels per precision.
  __shared__ uint64_t qa[KRR_MAX_GROUP], qb[KRR_MAX_GROUP];
  __shared__ int qp[KRR_MAX_GROUP], qsa[KRR_MAX_GROUP], qsb[KRR_MAX_GROUP];
  if (threadIdx.x < npan) {
    const int q = threadIdx.x, k = k0 + q;
    const int64_t a = i - k - 1, b = j - k - 1;
    int prec = KRR_PREC_FP32;
    if (i != j && pol.mode == KRR_POLICY_FIXED_MAP) {
      prec = pol.fmap[(int64_t)k * ntiles_all + i * (i + 1) / 2 + j];
      prec = prec > KRR_PREC_FP8 ? KRR_PREC_FP32 : prec;
    } else if (i != j && k >= pol.high_panels) {
      if (pol.mode == KRR_POLICY_FIXED) {
        prec = pol.fixed_prec;
      } else if (pol.mode == KRR_POLICY_ADAPTIVE) {
        // operand rule u_p ||L_ik|| ||L_jk|| <= thr, tile rule u_p ||A_ij|| <= thr,
        // or the lower precision of the two (the tile rule as a ceiling)
        double prod = (double)ps.pnorm[q][a] * (double)ps.pnorm[q][b];
        if (pol.rule == KRR_RULE_TILE) prod = pol.tnorm[i * (i + 1) / 2 + j];
        else if (pol.rule == KRR_RULE_BOTH) prod = fmax(prod, pol.tnorm[i * (i + 1) / 2 + j]);
        prec = rule_prec(pol, prod);
      }
    }
    // the panel's promotion cap and the precisions the attempt makes available
    prec = effective_prec(pol, k, prec);
    const int64_t ra = a * te + (int64_t)si * BM * nb, rb = b * te + (int64_t)sj * BM * nb;
    if (prec == KRR_PREC_FP32) {
      qa[q] = (uint64_t)(ps.P32[q] + ra);
      qb[q] = (uint64_t)(ps.P32[q] + rb);
    } else if (prec == KRR_PREC_FP16) {
      qa[q] = (uint64_t)(ps.P16[q] + ra);
      qb[q] = (uint64_t)(ps.P16[q] + rb);
    } else {
      qa[q] = (uint64_t)(ps.P8[q] + ra);
      qb[q] = (uint64_t)(ps.P8[q] + rb);
      qsa[q] = 127 - ps.pexp8[q][a];
      qsb[q] = 127 - ps.pexp8[q][b];
    }
    qp[q] = prec;
    if (first_sub) pmap[(int64_t)k * ntiles_all + i * (i + 1) / 2 + j] = (uint8_t)prec;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int cnt[3] = {0, 0, 0};
    for (int q = 0; q < npan; ++q) {
      const int p = qp[q], c = cnt[p]++;
      tab.a[p][c] = qa[q];
      tab.b[p][c] = qb[q];
      if (p == KRR_PREC_FP8) {
        tab.sa[c] = qsa[q];
        tab.sb[c] = qsb[q];
      }
    }
    tab.cnt[0] = cnt[0];
    tab.cnt[1] = cnt[1];
    tab.cnt[2] = cnt[2];
  }
  __syncthreads();
  const int c32 = __builtin_amdgcn_readfirstlane(tab.cnt[0]);
  const int c16 = __builtin_amdgcn_readfirstlane(tab.cnt[1]);
  const int c8 = __builtin_amdgcn_readfirstlane(tab.cnt[2]);
  // slabs (64 bytes of K) per panel: nb * element size / 64
  const int sh8 = 31 - __builtin_clz(nb / 64);

  OpF32::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  if (c32 > 0)
    gemm_nt_stream<OpF32, S>(SegSrc<OpF32>{(LdsSegTable)&tab, 0, sh8 + 2}, (int64_t)nb * 4, BM,
                             (int64_t)nb * 4, BM, (int64_t)c32 * nb * 4, acc, lds);
  if (c16 > 0)
    gemm_nt_stream<OpF16, S>(SegSrc<OpF16>{(LdsSegTable)&tab, 1, sh8 + 1}, (int64_t)nb * 2, BM,
                             (int64_t)nb * 2, BM, (int64_t)c16 * nb * 2, acc, lds);
  if (c8 > 0)
    gemm_nt_stream<OpF8, S>(SegSrc<OpF8>{(LdsSegTable)&tab, 2, sh8}, (int64_t)nb, BM, (int64_t)nb, BM,
                            (int64_t)c8 * nb, acc, lds);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float *C = Astore + (i * (i + 1) / 2 + j) * te + (int64_t)si * BM * nb + sj * BM;
  // C -= acc by a plain read-modify-write, a block row of accumulators at a
  // time (the loads of a row in flight together): the events that order the
  // launches give each launch its tiles alone, and every element gets one
  // subtraction per launch.  (One FP32 atomic add per element in L2 instead
  // was measured 1 ms per step slower at n = 32768.)
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm) {
    float cv[S::WTN][16];
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e)
        cv[tn][e] = C[(int64_t)S::row(wave, tm, e, lane) * nb + S::col(wave, tn, lane)];
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int e = 0; e < 16; ++e)
        C[(int64_t)S::row(wave, tm, e, lane) * nb + S::col(wave, tn, lane)] = cv[tn][e] - acc[tm][tn][e];
  }
}

template <class S, bool DIAG>
__global__ __launch_bounds__(S::THREADS) void k_update(
    float *__restrict__ Astore, PanelSet ps, int k0, int npan, int jlo, int jhi, int NT, int nb,
    int SB, UpdatePolicy pol, uint8_t *__restrict__ pmap, int64_t ntiles_all) {
  update_body<S, DIAG>(Astore, ps, k0, npan, jlo, jhi, NT, nb, SB, pol, pmap, ntiles_all,
                       blockIdx.x, gridDim.x);
}

void launch_update(float *Astore, int k0, int npan, int jlo, int jhi, const TileLayout &L,
                   const UpdatePolicy &pol, FactorWork &w, const PanelBuf *const *pbs,
                   uint8_t *pmap, int which, hipStream_t s) {
  const int NT = L.nt;
  if (npan <= 0 || jlo > jhi || jlo >= NT) return;
  if (jhi > NT - 1) jhi = NT - 1;
  int64_t offdiag = 0;  // tiles (i, j), jlo <= j <= jhi, i > j
  if (jhi == NT - 1) {
    const int64_t T = NT - jlo;
    offdiag = T * (T - 1) / 2;
  } else {
    for (int j = jlo; j <= jhi; ++j) offdiag += NT - 1 - j;
  }
  PanelSet ps{};
  for (int q = 0; q < npan; ++q) {
    ps.P32[q] = pbs[q]->P32;
    ps.P16[q] = pbs[q]->P16;
    ps.P8[q] = pbs[q]->P8;
    ps.pnorm[q] = pbs[q]->pnorm;
    ps.pexp8[q] = pbs[q]->pexp8;
  }
  factor_kernel_attrs();
  if (which != UPD_OFFDIAG) {  // diagonal tiles first: they are the longest per block
    const int SB = L.nb / UpdDiag64::kBM;
    const int64_t blocks = (int64_t)(jhi - jlo + 1) * SB * (SB + 1) / 2;
    hipLaunchKernelGGL((k_update<UpdDiag64, true>), dim3((unsigned)blocks),
                       dim3(UpdDiag64::THREADS), UpdDiag64::LDS_BYTES, s, Astore, ps, k0,
                       npan, jlo, jhi, NT, L.nb, SB, pol, pmap, L.ntiles());
  }
  if (which == UPD_DIAG) return;
  if (offdiag > 0 && offdiag * 4 < 8 * 256) {
    // few tiles (the updates inside a panel group, on the critical path):
    // small blocks, several per CU, for latency
    const int SB = L.nb / UpdDiagStream::kBM;
    const int64_t blocks = offdiag * SB * SB;
    hipLaunchKernelGGL((k_update<UpdDiagStream, false>), dim3((unsigned)blocks),
                       dim3(UpdDiagStream::THREADS), UpdDiagStream::LDS_BYTES, s, Astore, ps, k0,
                       npan, jlo, jhi, NT, L.nb, SB, pol, pmap, L.ntiles());
  } else if (offdiag > 0) {
    const int SB = L.nb / UpdStream::kBM;
    const int64_t blocks = offdiag * SB * SB;
    hipLaunchKernelGGL((k_update<UpdStream, false>), dim3((unsigned)blocks), dim3(UpdStream::THREADS),
                       UpdStream::LDS_BYTES, s, Astore, ps, k0, npan, jlo, jhi, NT, L.nb, SB,
                       pol, pmap, L.ntiles());
  }
}

// ---------------------------------------------------------------------------
// Lockstep batch: the kernels above behind a table of instances
// (blockIdx.y = instance).  A workgroup with nothing to do for its instance
// at this step returns before any barrier.
KRR_DEV int slot_of(int k, int g) { return ((k / g) & 1) * g + k % g; }

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_load_b(const FactorJob *__restrict__ jobs, int k,
                                                      int nb) {
  const FactorJob &j = jobs[blockIdx.y];
  if (k >= j.nt) return;
  DiagUpdate du;
  du.npan = 0;
  du.pmap = nullptr;
  potrf_load_body<T>(j.Lst + tri_index(k, k) * nb * nb, (T *)j.W, nb, du, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_diag64_b(const FactorJob *__restrict__ jobs, int k,
                                                        int nb) {
  const FactorJob &j = jobs[blockIdx.y];
  if (k >= j.nt) return;
  const int64_t te = (int64_t)nb * nb, db = (int64_t)(nb / BS) * BS * BS;
  potrf_diag64_first<T>((const T *)j.W, (T *)j.WL + k * te, nb, (T *)j.Dinv + k * db, j.flag,
                        (int64_t)k * nb);
}

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_step_b(const FactorJob *__restrict__ jobs, int k,
                                                      int st, int nb) {
  const FactorJob &j = jobs[blockIdx.y];
  if (k >= j.nt) return;
  const int64_t te = (int64_t)nb * nb, db = (int64_t)(nb / BS) * BS * BS;
  potrf_step_body<T>((T *)j.W, (T *)j.WL + k * te, nb, st, (T *)j.Dinv + k * db, j.flag,
                     (int64_t)k * nb, blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsm_panel_b(const FactorJob *__restrict__ jobs, int k,
                                                      int nb, int parts, int g) {
  const FactorJob &j = jobs[blockIdx.y];
  const int RS = nb / TRSM_ROWS;
  if (k + 1 >= j.nt || (int)(blockIdx.x / RS) >= j.nt - 1 - k) return;
  const int64_t te = (int64_t)nb * nb, db = (int64_t)(nb / BS) * BS * BS;
  trsm_panel_body<T>(j.Lst, (const T *)j.WL + k * te, (const T *)j.Dinv + k * db, k, 0, nb, parts,
                     j.P32[slot_of(k, g)], j.pnorm_part, j.pmax_part, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_convert_panel_b(const FactorJob *__restrict__ jobs, int k,
                                                         int nb, int chunks, int parts, int need16,
                                                         int need8, int scale8, int g) {
  const FactorJob &j = jobs[blockIdx.y];
  if (k + 1 >= j.nt || (int64_t)(blockIdx.x / chunks) >= j.nt - 1 - k) return;
  const int sl = slot_of(k, g);
  convert_panel_body(j.P32[sl], j.Lst, j.P16[sl], j.P8[sl], j.pnorm_part, j.pmax_part, parts,
                     j.pnorm[sl], j.pexp8[sl], k, nb, chunks, need16, need8, scale8, blockIdx.x);
}

// Tile inverse of diagonal tile k (and L_kk, inv(L_kk) into the factor
// storage), then the panel as a product with it.
template <typename T>
__global__ void k_trtri_init_b(const FactorJob *__restrict__ jobs, int k, int nb) {
  const FactorJob &j = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= j.nt || e >= (int64_t)nb * nb) return;
  const int NB = nb / BS;
  const T *D = (const T *)j.Dinv + (int64_t)k * NB * BS * BS;
  const int r = (int)(e / nb), q = (int)(e % nb);
  ((T *)j.Winv)[e] = (r / BS == q / BS) ? D[(int64_t)(r / BS) * BS * BS + (r % BS) * BS + q % BS]
                                        : (T)0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_trtri_level_b(const FactorJob *__restrict__ jobs, int k,
                                                       int nb, int b, int step, int pairs) {
  const FactorJob &j = jobs[blockIdx.z / pairs];
  if (k >= j.nt) return;
  const int64_t te = (int64_t)nb * nb;
  trtri_level_body<T>((const T *)j.WL + k * te, (T *)j.Winv, (T *)j.Tmp, nb, b, step,
                      blockIdx.z % pairs, blockIdx.y, blockIdx.x);
}

template <typename T>
__global__ void k_potrf_store_b(const FactorJob *__restrict__ jobs, int k, int nb) {
  const FactorJob &j = jobs[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= j.nt || e >= (int64_t)nb * nb) return;
  const int64_t te = (int64_t)nb * nb;
  const int r = (int)(e / nb), q = (int)(e % nb);
  j.Lst[((int64_t)k * (k + 1) / 2 + k) * te + e] = (q <= r) ? (float)((const T *)j.WL)[k * te + e] : 0.0f;
  j.Linv[k * te + e] = (q <= r) ? (float)((const T *)j.Winv)[e] : 0.0f;
}

__global__ __launch_bounds__(256) void k_trsm_gemm_b(const FactorJob *__restrict__ jobs, int k,
                                                     int nb, int parts, int g) {
  const FactorJob &j = jobs[blockIdx.y];
  const int SB = nb / TrsmShape::kBM;
  const int64_t nblk = (int64_t)(j.nt - 1 - k) * SB * SB;
  if (k + 1 >= j.nt || (int64_t)blockIdx.x >= nblk) return;
  trsm_gemm_body(j.Lst, j.Linv + (int64_t)k * nb * nb, k, 0, nb, parts, j.P32[slot_of(k, g)],
                 j.pnorm_part, j.pmax_part, xcd_remap(blockIdx.x, nblk));
}

// The update of one instance: in-group (panel k0 onto the group's later
// columns) or the group's update (panels G0 = k0 .. onto every column right
// of the group), clipped to the instance's tile count.  Returns its block
// count (0 when it has none) and its arguments.
__host__ __device__ inline int64_t update_extent(int nt, int k, bool group, int g, int SB, bool diag,
                                          int &k0, int &npan, int &jlo, int &jhi) {
  k0 = k;
  if (!group) {
    const int G0 = (k / g) * g;
    if (k >= nt) return 0;
    if (diag) {  // panel k onto the group's later diagonal tiles
      npan = 1;
      jlo = k + 1;
      jhi = min(G0 + g, nt) - 1;
    } else {  // left-looking: column k+1 gets the group's panels G0 .. k at once
      k0 = G0;
      npan = k - G0 + 1;
      jlo = jhi = k + 1;
      if (k + 1 >= min(G0 + g, nt)) return 0;
    }
  } else {
    npan = min(g, nt - k0);
    jlo = min(k0 + g, nt);
    jhi = nt - 1;
    if (npan < 1) return 0;
  }
  if (jlo > jhi) return 0;
  if (diag) return (int64_t)(jhi - jlo + 1) * SB * (SB + 1) / 2;
  int64_t off = 0;
  if (jhi == nt - 1) {
    const int64_t T = nt - jlo;
    off = T * (T - 1) / 2;
  } else {
    for (int jj = jlo; jj <= jhi; ++jj) off += nt - 1 - jj;
  }
  return off * SB * SB;
}

template <class S, bool DIAG>
__global__ __launch_bounds__(S::THREADS) void k_update_b(const FactorJob *__restrict__ jobs, int k0,
                                                         int group, int g, int nb, int SB,
                                                         UpdatePolicy pol) {
  const FactorJob &j = jobs[blockIdx.y];
  int kf, npan, jlo, jhi;
  const int64_t nblk = update_extent(j.nt, k0, group != 0, g, SB, DIAG, kf, npan, jlo, jhi);
  if ((int64_t)blockIdx.x >= nblk) return;
  PanelSet ps;
  for (int q = 0; q < npan; ++q) {
    const int sl = slot_of(kf + q, g);
    ps.P32[q] = j.P32[sl];
    ps.P16[q] = j.P16[sl];
    ps.P8[q] = j.P8[sl];
    ps.pnorm[q] = j.pnorm[sl];
    ps.pexp8[q] = j.pexp8[sl];
  }
  pol.thr = j.thr;
  pol.tnorm = j.tnorm;
  update_body<S, DIAG>(j.Lst, ps, kf, npan, jlo, jhi, j.nt, nb, SB, pol, j.pmap, j.ntiles,
                       blockIdx.x, nblk);
}

template <typename T>
static void factor_lockstep_t(const FactorJob *jobs, const int *nts, int nj, int nb, int g,
                              const UpdatePolicy &pol, bool need16, bool need8, bool scale8,
                              hipStream_t s) {
  const int NB = nb / BS, parts = trsm_parts(nb);
  const int chunks = (int)((int64_t)nb * nb / CONV_CHUNK_B);
  int ntmax = 0;
  for (int b = 0; b < nj; ++b) ntmax = std::max(ntmax, nts[b]);
  factor_kernel_attrs();
  // updates as launch_update does them: diagonal tiles (64 x 64 blocks),
  // then the off-diagonal ones, small blocks when the batch has few tiles
  // in all (grids sized for the instance with the most)
  auto update = [&](int k0, bool group) {
    const int SBd = nb / UpdDiagStream::kBM, SBo = nb / UpdStream::kBM, SB64 = nb / UpdDiag64::kBM;
    int64_t md = 0, mo = 0, so = 0, mo_small = 0;
    int kf, npan, jlo, jhi;
    for (int b = 0; b < nj; ++b) {
      md = std::max(md, update_extent(nts[b], k0, group, g, SB64, true, kf, npan, jlo, jhi));
      const int64_t off = update_extent(nts[b], k0, group, g, 1, false, kf, npan, jlo, jhi);
      mo = std::max(mo, off);
      so += off;
    }
    if (md > 0)
      hipLaunchKernelGGL((k_update_b<UpdDiag64, true>), dim3((unsigned)md, nj),
                         dim3(UpdDiag64::THREADS), UpdDiag64::LDS_BYTES, s, jobs, k0,
                         group ? 1 : 0, g, nb, SB64, pol);
    if (mo <= 0) return;
    if (so * 4 < 8 * 256) {
      mo_small = mo * SBd * SBd;
      hipLaunchKernelGGL((k_update_b<UpdDiagStream, false>), dim3((unsigned)mo_small, nj),
                         dim3(UpdDiagStream::THREADS), UpdDiagStream::LDS_BYTES, s, jobs, k0,
                         group ? 1 : 0, g, nb, SBd, pol);
    } else {
      hipLaunchKernelGGL((k_update_b<UpdStream, false>), dim3((unsigned)(mo * SBo * SBo), nj),
                         dim3(UpdStream::THREADS), UpdStream::LDS_BYTES, s, jobs, k0,
                         group ? 1 : 0, g, nb, SBo, pol);
    }
  };
  for (int G0 = 0; G0 < ntmax; G0 += g) {
    const int gend = std::min(G0 + g, ntmax);
    for (int k = G0; k < gend; ++k) {
      hipLaunchKernelGGL(k_potrf_load_b<T>, dim3(NB * (NB + 1) / 2, nj), dim3(256), 0, s, jobs, k,
                         nb);
      hipLaunchKernelGGL(k_potrf_diag64_b<T>, dim3(1, nj), dim3(256), 0, s, jobs, k, nb);
      for (int st = 0; st + 1 < NB; ++st) {
        const int rest = NB - 1 - st;
        hipLaunchKernelGGL(k_potrf_step_b<T>, dim3(rest * (rest + 1) / 2, nj), dim3(256), 0, s,
                           jobs, k, st, nb);
      }
      // inv(L_kk), then the panel as a product with it
      const unsigned eb = (unsigned)(((int64_t)nb * nb + 255) / 256);
      hipLaunchKernelGGL(k_trtri_init_b<T>, dim3(eb, nj), dim3(256), 0, s, jobs, k, nb);
      for (int b = BS; b < nb; b *= 2) {
        const unsigned nbk = (unsigned)(b / BS);
        const int pairs = nb / (2 * b);
        for (int step = 0; step < 2; ++step)
          hipLaunchKernelGGL(k_trtri_level_b<T>, dim3(nbk, nbk, pairs * nj), dim3(256), 0, s, jobs,
                             k, nb, b, step, pairs);
      }
      hipLaunchKernelGGL(k_potrf_store_b<T>, dim3(eb, nj), dim3(256), 0, s, jobs, k, nb);
      if (k + 1 < ntmax) {
        const int SBt = nb / TrsmShape::kBM;
        hipLaunchKernelGGL(k_trsm_gemm_b, dim3((unsigned)((ntmax - 1 - k) * SBt * SBt), nj),
                           dim3(256), 0, s, jobs, k, nb, parts, g);
        hipLaunchKernelGGL(k_convert_panel_b, dim3((unsigned)((int64_t)(ntmax - 1 - k) * chunks), nj),
                           dim3(256), 0, s, jobs, k, nb, chunks, parts, need16 ? 1 : 0,
                           need8 ? 1 : 0, scale8 ? 1 : 0, g);
      }
      update(k, false);
    }
    update(G0, true);
  }
}

void launch_factor_lockstep(const FactorJob *jobs, const int *nts, int njobs, int nb, int g,
                            const UpdatePolicy &pol, bool fp64, bool need16, bool need8,
                            bool scale8, hipStream_t s) {
  if (fp64)
    factor_lockstep_t<double>(jobs, nts, njobs, nb, g, pol, need16, need8, scale8, s);
  else
    factor_lockstep_t<float>(jobs, nts, njobs, nb, g, pol, need16, need8, scale8, s);
}

// Updates per operand precision, from the precision map (255 = no update).
__global__ void k_count_pmap(const uint8_t *__restrict__ pmap, int64_t n,
                             unsigned long long *counts) {
  unsigned long long c[3] = {0, 0, 0};
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int v = pmap[e];
    if (v < 3) c[v]++;
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    unsigned long long v = c[q];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(&counts[q], v);
  }
}

void launch_count_pmap(const uint8_t *pmap, int64_t n, unsigned long long *counts,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_count_pmap, dim3(256), dim3(256), 0, s, pmap, n, counts);
}

// Test hook: the factorization's FP8 encoder applied elementwise.
__global__ void k_encode_fp8(const float *__restrict__ x, int64_t n, uint8_t *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = f32_to_e4m3(x[e]);
}

void launch_encode_fp8(const float *x, int64_t n, uint8_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_encode_fp8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, out);
}

// Dynamic-LDS limits of the update kernels (above the 64 KB default), set once
// per process before their first launch; the context's creation calls it, so
// that it never runs inside a stream capture.
void factor_kernel_attrs() {
  static bool done = false;
  if (done) return;
  done = true;
  (void)hipFuncSetAttribute((const void *)k_update<UpdStream, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, UpdStream::LDS_BYTES);
  (void)hipFuncSetAttribute((const void *)k_update<UpdDiag64, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, UpdDiag64::LDS_BYTES);
  (void)hipFuncSetAttribute((const void *)k_update<UpdDiagStream, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, UpdDiagStream::LDS_BYTES);
  (void)hipFuncSetAttribute((const void *)k_update_b<UpdStream, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, UpdStream::LDS_BYTES);
  (void)hipFuncSetAttribute((const void *)k_update_b<UpdDiag64, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, UpdDiag64::LDS_BYTES);
  (void)hipFuncSetAttribute((const void *)k_update_b<UpdDiagStream, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, UpdDiagStream::LDS_BYTES);
}

}  // namespace krr
