// Shared device helpers for the gfx950 kernels of the KRR library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define KRR_DEV __device__ __forceinline__

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// Packed lower-triangle tile storage: tile (I, J), I >= J, is an nb x nb
// row-major block at tile index I (I + 1) / 2 + J.
KRR_DEV int64_t tri_index(int64_t I, int64_t J) { return I * (I + 1) / 2 + J; }

// Decode a linear index t over the lower triangle {(a, b): 0 <= b <= a}.
KRR_DEV void tri_decode(int64_t t, int &a, int &b) {
  int64_t x = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while (x * (x + 1) / 2 > t) --x;
  while ((x + 1) * (x + 2) / 2 <= t) ++x;
  a = (int)x;
  b = (int)(t - x * (x + 1) / 2);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap the hardware block id so that consecutive logical blocks --
// the sub-blocks of one output tile, which share operand rows -- run on the
// same XCD.
KRR_DEV int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  const int64_t per = nblocks / 8;
  if (per == 0 || bid >= per * 8) return bid;
  return (bid % 8) * per + bid / 8;
}

// ---------------------------------------------------------------------------
// OCP FP8 E4M3FN encoding (bias 7, max finite 448, no infinities), round to
// nearest even, saturating at +-448.  Written from the format definition.
KRR_DEV uint8_t f32_to_e4m3(float x) {
  const uint32_t sign = (__float_as_uint(x) >> 31) << 7;
  float a = fabsf(x);
  if (!(a < 448.0f)) return (uint8_t)(sign | 0x7E);  // saturate (NaN too)
  if (a <= 0x1p-10f) return (uint8_t)sign;           // at most half the least subnormal: +-0
  int e;
  frexpf(a, &e);      // a = f * 2^e, f in [0.5, 1)
  e -= 1;             // a = m * 2^e, m in [1, 2)
  if (e < -6) {       // subnormal range: multiples of 2^-9
    const float q = rintf(a * 512.0f);  // 0..8 (8 = smallest normal)
    return (uint8_t)(sign | (uint32_t)q);
  }
  float q = rintf(ldexpf(a, -e) * 8.0f) - 8.0f;  // mantissa steps of 1/8
  if (q >= 8.0f) { q = 0.0f; e += 1; }
  uint32_t code = ((uint32_t)(e + 7) << 3) | (uint32_t)q;
  if (code > 0x7E) code = 0x7E;
  return (uint8_t)(sign | code);
}

// Largest power of two s with maxabs * s <= limit (1 if maxabs is 0).
KRR_DEV float pow2_scale(float maxabs, float limit) {
  if (!(maxabs > 0.0f)) return 1.0f;
  int e;
  frexpf(limit / maxabs, &e);  // limit/maxabs = f * 2^e, f in [0.5,1)
  return ldexpf(1.0f, e - 1);
}

// ---------------------------------------------------------------------------
// Operand traits for the MFMA NT-GEMM core.  Every operand is row-major with
// the reduction dimension contiguous ("K-contiguous" on both sides).  The
// LDS slab is 64 bytes of K per row; each lane of a 32-lane half reads the
// 32 contiguous bytes at offset 32*half of its row.  A and B fragments use
// the same byte-to-k assignment, so each MFMA sums over a set of k that is
// the same for both operands and the slab's MFMAs cover all 64 bytes once:
// the product is exact regardless of the instruction's internal k order.

struct OpI8 {  // int8 x int8 -> int32 (v_mfma_i32_32x32x32_i8)
  typedef int8_t elem;
  typedef v16i acc_t;
  static constexpr int ebytes = 1;
  KRR_DEV void mma(acc_t &c, const v4i &a0, const v4i &a1, const v4i &b0, const v4i &b1) const {
    c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, c, 0, 0, 0);
  }
};

struct OpF16 {  // fp16 x fp16 -> fp32 (v_mfma_f32_32x32x16_f16)
  typedef _Float16 elem;
  typedef v16f acc_t;
  static constexpr int ebytes = 2;
  KRR_DEV void mma(acc_t &c, const v4i &a0, const v4i &a1, const v4i &b0, const v4i &b1) const {
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a0), __builtin_bit_cast(v8h, b0), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a1), __builtin_bit_cast(v8h, b1), c, 0, 0, 0);
  }
};

// OCP fp8 e4m3 x e4m3 -> fp32 (v_mfma_scale_f32_32x32x64_f8f6f4).  The
// operands are stored multiplied by powers of two; sa / sb are the E8M0
// exponents (127 + e means 2^e) that undo them inside the instruction.
struct OpF8 {
  typedef uint8_t elem;
  typedef v16f acc_t;
  static constexpr int ebytes = 1;
  int sa = 127, sb = 127;
  KRR_DEV void mma(acc_t &c, const v4i &a0, const v4i &a1, const v4i &b0, const v4i &b1) const {
    v8i a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
    v8i b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
    // format 0 = E4M3 for both operands
    c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, sa, 0, sb);
  }
};

struct OpF32 {  // fp32 x fp32 -> fp32 (v_mfma_f32_32x32x2f32, 8 per slab)
  typedef float elem;
  typedef v16f acc_t;
  static constexpr int ebytes = 4;
  KRR_DEV void mma(acc_t &c, const v4i &a0, const v4i &a1, const v4i &b0, const v4i &b1) const {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a0[e]), __int_as_float(b0[e]), c, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e)
      c = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a1[e]), __int_as_float(b1[e]), c, 0, 0, 0);
  }
};

// Output layout of a 32x32 MFMA accumulator: lane l, register i holds
// row 8*(i/4) + 4*(l/32) + (i%4), column l%32.
KRR_DEV int mfma_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }
KRR_DEV int mfma_col(int lane) { return lane & 31; }

// ---------------------------------------------------------------------------
// NT-GEMM core: acc[BM x BN] += A[BM x K] * B[BN x K]^T for one workgroup of
// WGM x WGN waves; each wave owns a (BM/WGM) x (BN/WGN) block of 32x32 MFMA
// tiles.  A and B are row-major with byte leading dimensions lda/ldb
// (multiples of 16) and K given in bytes (kbytes).  Rows at or beyond
// arows/brows, and bytes at or beyond kbytes, read as zero.  K is staged
// through LDS in 64-byte slabs, double-buffered, with the next slab's global
// loads issued before the current slab's MFMAs.
template <int BM, int BN, int WGM = 2, int WGN = 2, int SLABS = 1>
struct GemmShape {
  static constexpr int kBM = BM, kBN = BN, kWGM = WGM, kWGN = WGN, kSLABS = SLABS;
  static constexpr int THREADS = 64 * WGM * WGN;
  static constexpr int WROWS = BM / WGM;        // rows per wave
  static constexpr int WCOLS = BN / WGN;        // cols per wave
  static constexpr int WTM = WROWS / 32;        // MFMA tiles per wave, rows
  static constexpr int WTN = WCOLS / 32;        // MFMA tiles per wave, cols
  static constexpr int KB = 64 * SLABS;         // K bytes per pipeline stage
  static constexpr int ROWB = KB + 16;          // LDS row stride (bytes), padded
  static constexpr int STAGE = (BM + BN) * ROWB;
  static constexpr int LDS_BYTES = 2 * STAGE;
  static constexpr int CPR = KB / 16;           // 16-byte chunks per row per stage
  static constexpr int LA = BM * CPR / THREADS; // 16-byte loads per thread, A
  static constexpr int LB = BN * CPR / THREADS; // 16-byte loads per thread, B
  static_assert(LA * THREADS == BM * CPR && LB * THREADS == BN * CPR, "load split");
  // row / column (within the block) of accumulator register i of tile (tm, tn)
  KRR_DEV static int row(int wave, int tm, int i, int lane) {
    return (wave / WGN) * WROWS + tm * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
  }
  KRR_DEV static int col(int wave, int tn, int lane) {
    return (wave % WGN) * WCOLS + tn * 32 + (lane & 31);
  }
};

KRR_DEV v4i mask_tail(v4i v, int64_t keep) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t valid = keep - 4 * q;
    if (valid <= 0) v[q] = 0;
    else if (valid < 4) v[q] &= (int)((1u << (8 * valid)) - 1u);
  }
  return v;
}

template <class Op, class S>
KRR_DEV void gemm_nt_core(const Op &op, const uint8_t *__restrict__ A, int64_t lda, int arows,
                          const uint8_t *__restrict__ B, int64_t ldb, int brows, int64_t kbytes,
                          typename Op::acc_t (&acc)[S::WTM][S::WTN], uint8_t *lds) {
  constexpr int BM = S::kBM, BN = S::kBN, T = S::THREADS;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / S::kWGN, wn = wave % S::kWGN;

  // global load assignment: thread handles 16-byte chunk c of row r
  constexpr int CPR = S::CPR, KB = S::KB;
  v4i ra[S::LA], rb[S::LB];
  const int64_t nslab = (kbytes + KB - 1) / KB;

  auto gload = [&](int64_t slab) {
    const int64_t k0 = slab * KB;
#pragma unroll
    for (int t = 0; t < S::LA; ++t) {
      const int idx = tid + t * T;
      const int r = idx / CPR, c = idx % CPR;
      const int64_t kb = k0 + c * 16;
      v4i v = {0, 0, 0, 0};
      if (r < arows && kb < kbytes) {
        v = *(const v4i *)(A + (int64_t)r * lda + kb);
        if (kb + 16 > kbytes) v = mask_tail(v, kbytes - kb);
      }
      ra[t] = v;
    }
#pragma unroll
    for (int t = 0; t < S::LB; ++t) {
      const int idx = tid + t * T;
      const int r = idx / CPR, c = idx % CPR;
      const int64_t kb = k0 + c * 16;
      v4i v = {0, 0, 0, 0};
      if (r < brows && kb < kbytes) {
        v = *(const v4i *)(B + (int64_t)r * ldb + kb);
        if (kb + 16 > kbytes) v = mask_tail(v, kbytes - kb);
      }
      rb[t] = v;
    }
  };
  auto sstore = [&](int buf) {
    uint8_t *base = lds + buf * S::STAGE;
#pragma unroll
    for (int t = 0; t < S::LA; ++t) {
      const int idx = tid + t * T;
      const int r = idx / CPR, c = idx % CPR;
      *(v4i *)(base + r * S::ROWB + c * 16) = ra[t];
    }
    uint8_t *bb = base + BM * S::ROWB;
#pragma unroll
    for (int t = 0; t < S::LB; ++t) {
      const int idx = tid + t * T;
      const int r = idx / CPR, c = idx % CPR;
      *(v4i *)(bb + r * S::ROWB + c * 16) = rb[t];
    }
  };

  const int lrow = lane & 31, lhalf = lane >> 5;
  if (nslab > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int64_t s = 0; s < nslab; ++s) {
    const int buf = (int)(s & 1);
    if (s + 1 < nslab) gload(s + 1);
    const uint8_t *sa = lds + buf * S::STAGE;
    const uint8_t *sb = sa + BM * S::ROWB;
#pragma unroll
    for (int sl = 0; sl < S::kSLABS; ++sl) {
      v4i bf0[S::WTN], bf1[S::WTN];
#pragma unroll
      for (int tn = 0; tn < S::WTN; ++tn) {
        const uint8_t *p = sb + (wn * S::WCOLS + tn * 32 + lrow) * S::ROWB + sl * 64 + lhalf * 32;
        bf0[tn] = *(const v4i *)p;
        bf1[tn] = *(const v4i *)(p + 16);
      }
#pragma unroll
      for (int tm = 0; tm < S::WTM; ++tm) {
        const uint8_t *p = sa + (wm * S::WROWS + tm * 32 + lrow) * S::ROWB + sl * 64 + lhalf * 32;
        const v4i a0 = *(const v4i *)p;
        const v4i a1 = *(const v4i *)(p + 16);
#pragma unroll
        for (int tn = 0; tn < S::WTN; ++tn) op.mma(acc[tm][tn], a0, a1, bf0[tn], bf1[tn]);
      }
    }
    if (s + 1 < nslab) sstore(buf ^ 1);
    __syncthreads();
  }
  (void)BN;
}

template <class AccT, int WTM, int WTN>
KRR_DEV void zero_acc(AccT (&acc)[WTM][WTN]) {
#pragma unroll
  for (int a = 0; a < WTM; ++a)
#pragma unroll
    for (int b = 0; b < WTN; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0;
}

// Fixed-order block reduction of one double per thread (NW waves): wave
// butterfly, then the wave sums in index order.  Result valid in all threads.
template <int NW = 4>
KRR_DEV double block_sum(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r += sh[w];
  __syncthreads();
  return r;
}

template <int NW = 4>
KRR_DEV float block_max(float v, float *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = sh[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) r = fmaxf(r, sh[w]);
  __syncthreads();
  return r;
}
