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

// exp(-gamma d) for an integer distance d as the product of two table
// entries, exp(-gamma 512 hi) exp(-gamma lo) with d = 512 hi + lo: two small
// FP64 tables that fit in LDS (4m + 1 <= 512 * EXP_HI_MAX).  The product of
// the two correctly rounded factors is within two FP64 ulps of exp(-gamma d).
constexpr int EXP_LO = 512;         // entries of the low table
constexpr int EXP_HI_MAX = 2048;    // largest high table kept in LDS
KRR_DEV double exp_two_level(const double *hi, const double *lo, int32_t d) {
  return hi[d / EXP_LO] * lo[d % EXP_LO];
}

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
  static constexpr int ebytes = 1, NMMA = 2;  // MFMA instructions per mma()
  KRR_DEV void mma(acc_t &c, const v4i &a0, const v4i &a1, const v4i &b0, const v4i &b1) const {
    c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a0, b0, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_i32_32x32x32_i8(a1, b1, c, 0, 0, 0);
  }
};

struct OpF16 {  // fp16 x fp16 -> fp32 (v_mfma_f32_32x32x16_f16)
  typedef _Float16 elem;
  typedef v16f acc_t;
  static constexpr int ebytes = 2, NMMA = 2;
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
  static constexpr int ebytes = 1, NMMA = 1;
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
  static constexpr int ebytes = 4, NMMA = 8;
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

// ---------------------------------------------------------------------------
// Streamed NT-GEMM core, same product as gemm_nt_core, for large blocks.
// Full 64-byte K slabs go global -> LDS by direct-to-LDS loads
// (global_load_lds_dwordx4: lane l of an instruction fills bytes 16l .. 16l+15
// of a 1 KiB LDS run, no register staging) into an NST-deep ring; a partial
// last slab goes through registers with zero fill.  LDS rows are 64 bytes,
// unpadded: 16-byte chunk c of row r sits at chunk position c ^ swz(r), which
// puts the fragment reads of 8 or 16 consecutive rows on distinct banks.
// Each wave double-buffers its MFMA fragments (slab s+1 is read from LDS
// while the MFMAs of slab s run); one barrier per slab.
//
// Rows at or beyond arows / brows are read as copies of the last valid row:
// they only feed accumulator rows / columns that the caller discards.
template <int BM, int BN, int WGM, int WGN, int NST>
struct StreamShape {
  static constexpr int kBM = BM, kBN = BN, kWGM = WGM, kWGN = WGN, kNST = NST;
  static constexpr int THREADS = 64 * WGM * WGN, NWAVE = WGM * WGN;
  static constexpr int WROWS = BM / WGM, WCOLS = BN / WGN;
  static constexpr int WTM = WROWS / 32, WTN = WCOLS / 32;
  static constexpr int STAGE = (BM + BN) * 64;          // bytes per ring stage
  static constexpr int LDS_BYTES = NST * STAGE;
  static constexpr int LPW = (BM + BN) / 16 / NWAVE;    // 1 KiB loads per wave per slab
  static_assert(LPW * 16 * NWAVE == BM + BN && BM % 32 == 0 && BN % 32 == 0, "shape");
  static_assert(NST >= 2 && (NST - 2) * LPW <= 63, "ring depth");
  KRR_DEV static int row(int wave, int tm, int i, int lane) {
    return (wave / WGN) * WROWS + tm * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
  }
  KRR_DEV static int col(int wave, int tn, int lane) {
    return (wave % WGN) * WCOLS + tn * 32 + (lane & 31);
  }
};

KRR_DEV int lds_swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

// Counter waits and the workgroup barrier of the streamed core, as inline
// assembly with a memory clobber: the compiler may neither drop the waits nor
// move memory operations across them (a fenced __syncthreads() would instead
// wait for every direct-to-LDS load in flight).
// Wait until at most N of this wave's vector-memory operations are pending.
template <int N>
KRR_DEV void vm_wait() {
  static_assert(N >= 0 && N < 64, "vmcnt");
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
  __builtin_amdgcn_sched_barrier(0);
}
// Barrier after this wave's LDS reads and writes have completed.
KRR_DEV void bar_nofence() {
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// Instruction order of one streamed step, for the compiler's scheduler: one
// MFMA, then one LDS fragment read, while both last; then one MFMA and one
// direct load; then the MFMAs left.  Left to itself the scheduler puts every
// fragment read after the step's last MFMA, so the next step's barrier waits
// for all of the workgroup's LDS reads after its MFMAs instead of while they
// run.  (Masks: 0x008 MFMA, 0x100 LDS read, 0x060 vector memory.)
#ifndef KRR_GEMM_SCHED
#define KRR_GEMM_SCHED 1
#endif
template <int NMM, int NDS, int NVM>
KRR_DEV void sched_interleave() {
#if KRR_GEMM_SCHED
  constexpr int P = NMM < NDS ? NMM : NDS;
  constexpr int Q = NMM - P < NVM ? NMM - P : NVM;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  if (NDS > P) __builtin_amdgcn_sched_group_barrier(0x100, NDS - P, 0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x060, 1, 0);
  }
  if (NVM > Q) __builtin_amdgcn_sched_group_barrier(0x060, NVM - Q, 0);
  if (NMM > P + Q) __builtin_amdgcn_sched_group_barrier(0x008, NMM - P - Q, 0);
#endif
}

// K source of one product: ptr(side_a, s) is the address of slab s (64 bytes
// of K) in row 0 of A (side_a) or of B; op(s) is the MFMA operation for slab
// s.  Both are branch-free.  Plain contiguous operands:
template <class Op>
struct ContigSrc {
  const uint8_t *A, *B;
  Op o;
  KRR_DEV const uint8_t *ptr(bool side_a, int64_t s) const { return (side_a ? A : B) + s * 64; }
  KRR_DEV Op op(int64_t) const { return o; }
};

template <class Op, class S, class Src>
KRR_DEV void gemm_nt_stream(const Src &src, int64_t lda, int arows, int64_t ldb, int brows,
                            int64_t kbytes, typename Op::acc_t (&acc)[S::WTM][S::WTN],
                            uint8_t *lds) {
  constexpr int BM = S::kBM, NST = S::kNST, LPW = S::LPW, WTM = S::WTM, WTN = S::WTN;
  static_assert(BM % (LPW * 16) == 0, "each wave loads rows of one operand only");
    typedef __attribute__((address_space(3))) void lds_void;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave / S::kWGN, wn = wave % S::kWGN;
  const int64_t nfull = kbytes >> 6;       // whole 64-byte slabs
  const int64_t nmain = nfull & ~(int64_t)1;  // pairs of them go through the ring
  const int64_t nslab = (kbytes + 63) >> 6;

  // rows this wave moves: 16 LPW consecutive rows of A (waves in front) or B
  const bool side_a = wave * LPW * 16 < BM;
  const int r0 = side_a ? wave * LPW * 16 : wave * LPW * 16 - BM;
  const int rows = side_a ? arows : brows;
  const int64_t ld = side_a ? lda : ldb;
  uint32_t off[LPW];
#pragma unroll
  for (int t = 0; t < LPW; ++t) {
    const int R = r0 + t * 16 + (lane >> 2);
    off[t] = (uint32_t)((int64_t)min(R, rows - 1) * ld) + 16u * ((lane & 3) ^ lds_swz(R));
  }
  // Direct loads of slab s into ring stage `slot`.  Issued unconditionally
  // (slabs past the last repeat it), so the number of loads in flight -- and
  // the counter waits -- never vary.
  auto issue = [&](int slot, int64_t s) {
    const uint8_t *base = src.ptr(side_a, s);
    uint8_t *dst = lds + slot * S::STAGE + wave * LPW * 1024;
#pragma unroll
    for (int t = 0; t < LPW; ++t)
      __builtin_amdgcn_global_load_lds((const void *)(base + off[t]), (lds_void *)(dst + t * 1024),
                                       16, 0, 0);
  };

  const int lrow = lane & 31, lhalf = lane >> 5, sw = lds_swz(lrow);
  const int off0 = lrow * 64 + 16 * ((2 * lhalf) ^ sw);
  const int off1 = lrow * 64 + 16 * ((2 * lhalf + 1) ^ sw);
  auto frag = [&](int stage, v4i (&a0)[WTM], v4i (&a1)[WTM], v4i (&b0)[WTN], v4i (&b1)[WTN]) {
    const uint8_t *base = lds + stage * S::STAGE;
#pragma unroll
    for (int tn = 0; tn < WTN; ++tn) {
      const uint8_t *p = base + (BM + wn * S::WCOLS + tn * 32) * 64;
      b0[tn] = *(const v4i *)(p + off0);
      b1[tn] = *(const v4i *)(p + off1);
    }
#pragma unroll
    for (int tm = 0; tm < WTM; ++tm) {
      const uint8_t *p = base + (wm * S::WROWS + tm * 32) * 64;
      a0[tm] = *(const v4i *)(p + off0);
      a1[tm] = *(const v4i *)(p + off1);
    }
  };
  auto mma_rows = [&](int tm0, int tm1, const Op &o, v4i (&a0)[WTM], v4i (&a1)[WTM],
                      v4i (&b0)[WTN], v4i (&b1)[WTN]) {
#pragma unroll
    for (int tm = tm0; tm < tm1; ++tm)
#pragma unroll
      for (int tn = 0; tn < WTN; ++tn) o.mma(acc[tm][tn], a0[tm], a1[tm], b0[tn], b1[tn]);
  };

  v4i xa0[WTM], xa1[WTM], xb0[WTN], xb1[WTN];  // fragments, even slabs
  v4i ya0[WTM], ya1[WTM], yb0[WTN], yb1[WTN];  // fragments, odd slabs
  if (nmain > 0) {
    const int64_t last = nmain - 1;
#pragma unroll
    for (int s = 0; s < NST; ++s) issue(s, min((int64_t)s, last));
    vm_wait<(NST - 1) * LPW>();  // slab 0 landed
    bar_nofence();
    frag(0, xa0, xa1, xb0, xb1);
    Op ox = src.op(0), oy = ox;
    // Slab s, fragments in (c*): once slab s+1 has landed everywhere (slabs
    // s+2 .. s+NST-1 may still be in flight) and every wave holds slab s in
    // registers, the direct loads of slab s+NST (into slab s's stage) and the
    // fragment reads of slab s+1 (into n*) are issued with the MFMAs of slab
    // s.  Nothing in the step branches.
    auto step = [&](int64_t s, const Op &co, v4i (&ca0)[WTM], v4i (&ca1)[WTM], v4i (&cb0)[WTN],
                    v4i (&cb1)[WTN], Op &no, v4i (&na0)[WTM], v4i (&na1)[WTM],
                    v4i (&nb0)[WTN], v4i (&nb1)[WTN]) {
      vm_wait<(NST - 2) * LPW>();
      bar_nofence();
      issue((int)(s % NST), min(s + NST, last));
      frag((int)((s + 1) % NST), na0, na1, nb0, nb1);
      no = src.op(min(s + 1, last));
      mma_rows(0, WTM, co, ca0, ca1, cb0, cb1);
      sched_interleave<WTM * WTN * Op::NMMA, 2 * (WTM + WTN), LPW>();
    };
    for (int64_t s = 0; s < nmain; s += 2) {
      step(s, ox, xa0, xa1, xb0, xb1, oy, ya0, ya1, yb0, yb1);
      // past the last pair this reads a repeated slab that is never used
      step(s + 1, oy, ya0, ya1, yb0, yb1, ox, xa0, xa1, xb0, xb1);
    }
    vm_wait<0>();  // no direct load may land after the ring is handed back
  }
  // odd last whole slab and partial slab: through registers, one at a time,
  // bytes past kbytes read as zero
  for (int64_t s = nmain; s < nslab; ++s) {
    const int valid = (int)min((int64_t)64, kbytes - s * 64);
    bar_nofence();  // every wave is past its reads of the ring
    const uint8_t *base = src.ptr(side_a, s);
    uint8_t *dst = lds + wave * LPW * 1024;
#pragma unroll
    for (int t = 0; t < LPW; ++t) {
      const int c16 = 16 * ((lane & 3) ^ lds_swz(lane >> 2));
      v4i v = {0, 0, 0, 0};
      if (c16 < valid) {
        v = *(const __attribute__((address_space(1))) v4i *)(base + off[t]);
        if (c16 + 16 > valid) v = mask_tail(v, valid - c16);
      }
      *(v4i *)(dst + t * 1024 + lane * 16) = v;
    }
    bar_nofence();
    frag(0, xa0, xa1, xb0, xb1);
    mma_rows(0, WTM, src.op(s), xa0, xa1, xb0, xb1);
  }
  bar_nofence();  // the ring is free for the caller's next use
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
