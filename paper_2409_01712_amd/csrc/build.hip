// Build phase: squared genotype distances through an INT8 MFMA Gram and the
// Gaussian kernel, per tile (arXiv 2409.01712, Algorithm 2 with the
// Gaussian kernel of Algorithm 5; "Engaging INT8 Tensor Cores for Distance
// Calculations" and "TC-based Distance Computations").
//
// d_ij = n_i + n_j - 2 <g_i, g_j> with the per-patient squared norms n_i kept
// as one vector (the paper's folded D), the Gram term from INT8 MFMA with
// int32 accumulation (exact: every partial sum is at most 4m), and each entry
// exponentiated before the tile leaves registers.  Only tiles I >= J of the
// symmetric matrix are computed.
#include "common.h"
#include "internal.h"

namespace krr {

// exp(-gamma * d) for every integer distance d in [0, len): the FP64 kernel
// value of any entry is then a table lookup, bit-identical to evaluating exp.
// The FP32 matrix handed to the factorization takes the value as the
// two-level product of common.h (exp_two_level), rounded to FP32 (within one
// FP32 ulp of the correctly rounded value).
__global__ void k_exp_table(double *tab, int64_t len, double gamma) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) tab[i] = exp(-gamma * (double)i);
}

void launch_exp_table(double *tab, int64_t len, double gamma, hipStream_t s) {
  const int64_t blocks = (len + 255) / 256;
  hipLaunchKernelGGL(k_exp_table, dim3((unsigned)blocks), dim3(256), 0, s, tab, len, gamma);
}

// Row norms n_i = sum_k g_ik^2 (one workgroup per row, 16-byte loads, dot4),
// and the genotype check: any byte outside {0, 1, 2} sets *flag.  Rows
// n .. rows_padded-1 are padding and get n_i = 0.
KRR_DEV void row_norm(const int8_t *__restrict__ G, int64_t n, int64_t m, int64_t ldg,
                      int32_t *nrm, int32_t *flag, int64_t row) {
  __shared__ int sh[4];
  if (row >= n) {
    if (threadIdx.x == 0) nrm[row] = 0;
    return;
  }
  const uint8_t *p = (const uint8_t *)G + row * ldg;
  uint32_t acc = 0, bad = 0;
  for (int64_t kb = (int64_t)threadIdx.x * 16; kb < m; kb += 256 * 16) {
    v4i v = *(const v4i *)(p + kb);
    const int64_t keep = m - kb;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t w = (uint32_t)v[q];
      const int64_t valid = keep - 4 * q;
      if (valid <= 0) w = 0;
      else if (valid < 4) w &= (1u << (8 * valid)) - 1u;
      bad |= (w & 0xFCFCFCFCu) | ((w & (w >> 1)) & 0x01010101u);
      acc = __builtin_amdgcn_udot4(w, w, acc, false);
    }
  }
  int s = (int)acc;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  if (threadIdx.x == 0) nrm[row] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(256) void k_row_norms(const int8_t *__restrict__ G, int64_t n,
                                                   int64_t m, int64_t ldg, int32_t *nrm,
                                                   int32_t *flag) {
  row_norm(G, n, m, ldg, nrm, flag, blockIdx.x);
}

void launch_row_norms(const int8_t *G, int64_t n, int64_t rows_padded, int64_t m, int64_t ldg,
                      int32_t *nrm, int32_t *flag, hipStream_t s) {
  hipLaunchKernelGGL(k_row_norms, dim3((unsigned)rows_padded), dim3(256), 0, s, G, n, m, ldg,
                     nrm, flag);
}

// The genotypes in slab-major order: slab s (bytes 64 s .. 64 s + 63 of every
// row) of all np rows one after another, Gs[(s np + r) 64 + b], zero past m
// and on the padding rows.  A block of the Gram then streams each slab of its
// 256 rows as one contiguous 16 KiB run (whole 128-byte lines) instead of 256
// runs of 64 bytes a row apart.
__global__ void k_slab_major(const int8_t *__restrict__ G, int64_t n, int64_t np, int64_t m,
                             int64_t ldg, int64_t nslab, int8_t *__restrict__ Gs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one 16-byte chunk
  if (e >= nslab * np * 4) return;
  const int c = (int)(e & 3);
  const int64_t r = (e >> 2) % np, sl = (e >> 2) / np, kb = sl * 64 + 16 * c;
  v4i v = {0, 0, 0, 0};
  if (r < n && kb < m) {
    v = *(const v4i *)(G + r * ldg + kb);
    if (kb + 16 > m) v = mask_tail(v, m - kb);
  }
  *(v4i *)(Gs + e * 16) = v;
}

// The slab-major copy and the row norms (with the genotype check) in one
// pass over G: a workgroup takes 32 rows and a run of slab pairs, each row's
// 128 bytes of a pair read by eight threads (whole lines) and written to its
// two slabs; each thread sums the squares of its bytes over the run
// (udot4), the eight of a row add theirs and one atomic add per row and
// workgroup puts the sum into nrm (zeroed before: integer sums, so the order
// does not matter).  Bytes above 2 (not a genotype) set flag.
constexpr int SLAB_RUN = 64;  // slab pairs a workgroup
__global__ __launch_bounds__(256) void k_slab_major_norms(const int8_t *__restrict__ G, int64_t n,
                                                          int64_t np, int64_t m, int64_t ldg,
                                                          int64_t nslab, int8_t *__restrict__ Gs,
                                                          int32_t *__restrict__ nrm,
                                                          int32_t *flag) {
  const int tid = threadIdx.x, c = tid & 7;
  const int64_t r = (int64_t)blockIdx.x * 32 + (tid >> 3);
  const int64_t nsp = (nslab + 1) / 2, sp0 = (int64_t)blockIdx.y * SLAB_RUN;
  const int64_t sp1 = min(nsp, sp0 + SLAB_RUN);
  const int64_t slab_of = c >> 2, off = 16 * (c & 3);
  uint32_t acc = 0, bad = 0;
  for (int64_t sp = sp0; sp < sp1; sp += 8) {
    v4i v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t kb = (sp + u) * 128 + 16 * c;
      v[u] = (v4i){0, 0, 0, 0};
      if (sp + u < sp1 && r < n && kb < m) {
        v[u] = *(const v4i *)(G + r * ldg + kb);
        if (kb + 16 > m) v[u] = mask_tail(v[u], m - kb);
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t sl = 2 * (sp + u) + slab_of;
      if (sp + u < sp1 && sl < nslab && r < np) *(v4i *)(Gs + (sl * np + r) * 64 + off) = v[u];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t w = (uint32_t)v[u][q];
        bad |= (w & 0xFCFCFCFCu) | ((w & (w >> 1)) & 0x01010101u);
        acc = __builtin_amdgcn_udot4(w, w, acc, false);
      }
    }
  }
  int sum = (int)acc;
  sum += __shfl_xor(sum, 1, 64);
  sum += __shfl_xor(sum, 2, 64);
  sum += __shfl_xor(sum, 4, 64);
  if (c == 0 && r < n && sum != 0) atomicAdd(&nrm[r], sum);
  if (bad) atomicOr(flag, 1);
}

void launch_slab_major_norms(const int8_t *G, int64_t n, int64_t np, int64_t m, int64_t ldg,
                             int8_t *Gs, int32_t *nrm, int32_t *flag, hipStream_t s) {
  const int64_t nslab = (m + 63) / 64, nsp = (nslab + 1) / 2;
  launch_fill_i32(nrm, np, 0, s);
  hipLaunchKernelGGL(k_slab_major_norms,
                     dim3((unsigned)((np + 31) / 32), (unsigned)((nsp + SLAB_RUN - 1) / SLAB_RUN)),
                     dim3(256), 0, s, G, n, np, m, ldg, nslab, Gs, nrm, flag);
}

void launch_slab_major(const int8_t *G, int64_t n, int64_t np, int64_t m, int64_t ldg,
                       int8_t *Gs, hipStream_t s) {
  const int64_t nslab = (m + 63) / 64, cnt = nslab * np * 4;
  hipLaunchKernelGGL(k_slab_major, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, G, n, np,
                     m, ldg, nslab, Gs);
}

// K source over a slab-major matrix: slab s of rows ra .. (A) or rb .. (B),
// rows 64 bytes apart.
template <class Op>
struct SlabSrc {
  const uint8_t *Gs;
  int64_t np, ra, rb;
  Op o;
  KRR_DEV const uint8_t *ptr(bool side_a, int64_t s) const {
    return Gs + (s * np + (side_a ? ra : rb)) * 64;
  }
  KRR_DEV Op op(int64_t) const { return o; }
};

// Symmetric Gram over the lower tile triangle.  Block (BM x BN) = one
// sub-block of tile (I, J); SB x SB sub-blocks per tile.  Epilogue per
// entry: d = n_i + n_j - 2 S (int32), A = exp(-gamma d) (two-level table in
// LDS, FP64 product rounded to FP32), 1 + lambda on the diagonal, identity
// on padding; plus the sub-block's FP64 sum of squares for the tile norms.
// vmode (VAL_*): VAL_EXP the Gaussian through the exponential tables;
// VAL_TABLE another kernel of the distance held in the table (IBS), a plain
// lookup per entry; VAL_LINEAR the linear kernel: the Gram entry itself is
// stored and is the value.  Ec (or null): FP64 confounder factors
// exp(-gamma dc_ij) in the packed tile layout, multiplied in.
// Gs (or null): the same genotypes slab-major (k_slab_major), read instead of G.
// Block (bi, bj) -- 256-row blocks of the padded matrix -- that workgroup t
// computes in the grouped order: super-rows of GRP block rows, column by
// column within a super-row, the rows of one column consecutive.  The blocks
// computed are those with tile(bi) >= tile(bj), tile(b) = b / SB (the lower
// tiles, diagonal tiles whole).  The workgroups an XCD runs at one time then
// cover a GRP x 8 patch of blocks, reading GRP + 8 blocks of rows per K slab,
// in place of one block row of tiles (at tile 256: 1 + 32 blocks of rows).
constexpr int GRAM_GRP = 4;
KRR_DEV void gram_grouped(int64_t t, int nbk, int SB, int &bi, int &bj) {
  for (int r0 = 0; r0 < nbk; r0 += GRAM_GRP) {
    const int h = min(GRAM_GRP, nbk - r0);
    const int64_t full = (int64_t)r0 * h;  // columns left of the super-row: every row
    if (t < full) {
      bj = (int)(t / h);
      bi = r0 + (int)(t % h);
      return;
    }
    t -= full;
    const int cend = min(nbk, (r0 + h - 1) / SB * SB + SB);
    for (int c = r0; c < cend; ++c) {
      const int rfirst = max(r0, c / SB * SB);  // first row whose tile reaches column c's
      const int cnt = r0 + h - rfirst;
      if (t < cnt) {
        bj = c;
        bi = rfirst + (int)t;
        return;
      }
      t -= cnt;
    }
  }
  bi = bj = 0;  // t past the last block: not launched
}

template <class S>
KRR_DEV void gram_block(const int8_t *__restrict__ G, int64_t n, int64_t m, int64_t ldg,
                        const int32_t *__restrict__ nrm, const double *__restrict__ etab,
                        int64_t etab_len, double lambda, int nb, int SB, int32_t *__restrict__ D,
                        float *__restrict__ A, double *part, int64_t bid, int vmode,
                        const double *__restrict__ Ec, const int8_t *__restrict__ Gs = nullptr,
                        int64_t np = 0, bool grouped = false) {
  constexpr int BM = S::kBM, BN = S::kBN, NW = S::THREADS / 64;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  __shared__ double shd[NW];
  __shared__ double ehi[EXP_HI_MAX], elo[EXP_LO];
  const int64_t dmax = etab_len - 1;
  const int nhi = (int)(dmax / EXP_LO) + 1;
  const bool two_level = vmode == VAL_EXP && nhi <= EXP_HI_MAX;
  if (two_level) {  // visible to the epilogue through the GEMM's barriers
    for (int q = threadIdx.x; q < EXP_LO; q += S::THREADS) elo[q] = etab[min((int64_t)q, dmax)];
    for (int q = threadIdx.x; q < nhi; q += S::THREADS) ehi[q] = etab[(int64_t)q * EXP_LO];
  }
  const int nsub = SB * SB;
  int I, J, si, sj;
  if (grouped) {
    int bi, bj;
    gram_grouped(bid, (int)((n + nb - 1) / nb) * SB, SB, bi, bj);
    I = bi / SB, J = bj / SB, si = bi % SB, sj = bj % SB;
  } else {  // tiles in packed order, the sub-blocks of a tile consecutive
    tri_decode(bid / nsub, I, J);
    si = (int)(bid % nsub) / SB, sj = (int)(bid % nsub) % SB;
  }
  const int sub = si * SB + sj;
  const int64_t tt = tri_index(I, J);  // the tile's place in the packed storage
  const int64_t row0 = (int64_t)I * nb + si * BM, col0 = (int64_t)J * nb + sj * BN;
  const int arows = (int)max((int64_t)0, min((int64_t)BM, n - row0));
  const int brows = (int)max((int64_t)0, min((int64_t)BN, n - col0));

  OpI8::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  if (arows > 0 && brows > 0) {
    if (Gs)
      gemm_nt_stream<OpI8, S>(SlabSrc<OpI8>{(const uint8_t *)Gs, np, row0, col0, OpI8{}}, 64,
                              arows, 64, brows, ((m + 63) / 64) * 64, acc, lds);
    else
      gemm_nt_stream<OpI8, S>(
          ContigSrc<OpI8>{(const uint8_t *)G + row0 * ldg, (const uint8_t *)G + col0 * ldg,
                          OpI8{}},
          ldg, arows, ldg, brows, m, acc, lds);
  }
  __syncthreads();  // the tables (also when the product was skipped)

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t tbase = tt * (int64_t)nb * nb;
  double ss = 0.0;
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int r = S::row(wave, tm, i, lane);
        const int c = S::col(wave, tn, lane);
        const int64_t gi = row0 + r, gj = col0 + c;
        int32_t d;
        float a;
        const int64_t off = tbase + (int64_t)(si * BM + r) * nb + sj * BN + c;
        if (gi < n && gj < n && vmode == VAL_LINEAR) {
          d = acc[tm][tn][i];  // the inner product is the value (exact in FP32 below 2^24)
          a = (float)((double)d + (gi == gj ? lambda : 0.0));
        } else if (gi < n && gj < n) {
          d = nrm[gi] + nrm[gj] - 2 * acc[tm][tn][i];
          const int32_t dc = (int32_t)min((int64_t)max(d, 0), dmax);
          double e = two_level ? exp_two_level(ehi, elo, dc) : etab[dc];
          if (Ec) e *= Ec[off];
          a = (gi == gj) ? (float)(1.0 + lambda) : (float)e;
        } else {
          d = 0;
          a = (gi == gj) ? 1.0f : 0.0f;
        }
        D[off] = d;
        A[off] = a;
        ss += (double)a * (double)a;
      }
  ss = block_sum<NW>(ss, shd);
  if (threadIdx.x == 0) part[tt * nsub + sub] = ss;
}

template <class S>
__global__ __launch_bounds__(S::THREADS) void k_gram_tiles(const int8_t *__restrict__ G, int64_t n,
                                                    int64_t m, int64_t ldg,
                                                    const int32_t *__restrict__ nrm,
                                                    const double *__restrict__ etab,
                                                    int64_t etab_len, double lambda, int nb,
                                                    int SB, int32_t *__restrict__ D,
                                                    float *__restrict__ A, double *part,
                                                    int vmode,
                                                    const double *__restrict__ Ec,
                                                    const int8_t *__restrict__ Gs, int64_t np,
                                                    int grouped) {
  gram_block<S>(G, n, m, ldg, nrm, etab, etab_len, lambda, nb, SB, D, A, part,
                xcd_remap(blockIdx.x, gridDim.x), vmode, Ec, Gs, np, grouped != 0);
}

// Instance of a batch that owns workgroup `bid`: the last job whose first
// workgroup (field F of BuildJob) is <= bid.
template <int64_t BuildJob::*F>
KRR_DEV int find_job(const BuildJob *jobs, int njobs, int64_t bid) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].*F <= bid) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// All instances of a batch in one launch: each workgroup finds its instance
// and runs the same block as the single-instance kernel.
template <class S>
__global__ __launch_bounds__(S::THREADS) void k_gram_tiles_batched(const BuildJob *__restrict__ jobs,
                                                            int njobs, int64_t m, int nb, int SB,
                                                            int grouped) {
  const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const BuildJob &j = jobs[find_job<&BuildJob::block0>(jobs, njobs, bid)];
  gram_block<S>(j.G, j.n, m, j.ldg, j.nrm, j.etab, j.etab_len, j.lambda, nb, SB, j.D, j.A, j.part,
                bid - j.block0, VAL_EXP, nullptr, nullptr, 0, grouped != 0);
}

typedef StreamShape<256, 256, 2, 4, 4> GramShape;

// The Gram's blocks in the grouped order, unless KRR_GRAM_ORDER=0 (tiles in
// packed order, for comparison).
static int gram_grouped_order() {
  static const int grouped = [] {
    const char *e = getenv("KRR_GRAM_ORDER");
    return (e && atoi(e) == 0) ? 0 : 1;
  }();
  return grouped;
}

void launch_gram_tiles(const int8_t *G, int64_t m, int64_t ldg, const int32_t *nrm,
                       const double *etab, int64_t etab_len, double lambda, const TileLayout &L,
                       int32_t *D, float *A, double *tnorm_part, int vmode,
                       const double *Ec, const int8_t *Gs, hipStream_t s) {
  const int SB = L.nb / GramShape::kBM;
  const int grouped = gram_grouped_order();
  const int64_t blocks = L.ntiles() * SB * SB;
  build_kernel_attrs();
  hipLaunchKernelGGL((k_gram_tiles<GramShape>), dim3((unsigned)blocks), dim3(GramShape::THREADS),
                     GramShape::LDS_BYTES, s, G, L.n, m,
                     ldg, nrm, etab, etab_len, lambda, L.nb, SB, D, A, tnorm_part, vmode, Ec, Gs,
                     L.np, grouped);
}

int64_t gram_blocks(const TileLayout &L) {
  const int SB = L.nb / GramShape::kBM;
  return L.ntiles() * SB * SB;
}

int gram_parts(int nb) { return (nb / GramShape::kBM) * (nb / GramShape::kBM); }

void launch_gram_tiles_batched(const BuildJob *jobs, int njobs, int64_t blocks, int64_t m, int nb,
                               hipStream_t s) {
  build_kernel_attrs();
  hipLaunchKernelGGL((k_gram_tiles_batched<GramShape>), dim3((unsigned)blocks),
                     dim3(GramShape::THREADS), GramShape::LDS_BYTES, s, jobs, njobs, m, nb,
                     nb / GramShape::kBM, gram_grouped_order());
}

__global__ __launch_bounds__(256) void k_row_norms_batched(const BuildJob *__restrict__ jobs,
                                                           int njobs, int64_t m) {
  const BuildJob &j = jobs[find_job<&BuildJob::row0>(jobs, njobs, blockIdx.x)];
  row_norm(j.G, j.n, m, j.ldg, j.nrm, j.flag, (int64_t)blockIdx.x - j.row0);
}

void launch_row_norms_batched(const BuildJob *jobs, int njobs, int64_t rows, int64_t m,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_row_norms_batched, dim3((unsigned)rows), dim3(256), 0, s, jobs, njobs, m);
}

__global__ void k_exp_tables_batched(const BuildJob *__restrict__ jobs) {
  const BuildJob &j = jobs[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < j.etab_len) j.etab[i] = exp(-j.gamma * (double)i);
}

void launch_exp_tables_batched(const BuildJob *jobs, int njobs, int64_t max_len, hipStream_t s) {
  hipLaunchKernelGGL(k_exp_tables_batched, dim3((unsigned)((max_len + 255) / 256), njobs),
                     dim3(256), 0, s, jobs);
}

__global__ void k_tile_norms_batched(const BuildJob *__restrict__ jobs, int parts) {
  const BuildJob &j = jobs[blockIdx.y];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= j.ntiles) return;
  double s = 0.0;
  for (int q = 0; q < parts; ++q) s += j.part[t * parts + q];
  j.tnorm[t] = sqrt(s);
}

void launch_tile_norms_batched(const BuildJob *jobs, int njobs, int64_t max_ntiles, int nb,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_tile_norms_batched, dim3((unsigned)((max_ntiles + 255) / 256), njobs),
                     dim3(256), 0, s, jobs, gram_parts(nb));
}

// Tile Frobenius norms from the per-sub-block partial sums, in fixed order.
__global__ void k_tile_norms(const double *part, int parts, int64_t ntiles, double *tnorm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  double s = 0.0;
  for (int q = 0; q < parts; ++q) s += part[t * parts + q];
  tnorm[t] = sqrt(s);
}

void launch_tile_norms(const double *part, int parts, int64_t ntiles, double *tnorm,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_tile_norms, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, s, part,
                     parts, ntiles, tnorm);
}

// Re-expand K + lambda*I from the stored distances (same values the Gram
// epilogue wrote), for a second factorization of one kernel.
__global__ void k_expand_tiles(const int32_t *__restrict__ D, const double *__restrict__ etab,
                               int64_t etab_len, double lambda, int64_t n, int nb, int64_t total,
                               int vmode, const double *__restrict__ Ec,
                               float *__restrict__ A) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t te = (int64_t)nb * nb;
  const int64_t t = e / te, w = e % te;
  int I, J;
  tri_decode(t, I, J);
  const int64_t gi = (int64_t)I * nb + w / nb, gj = (int64_t)J * nb + w % nb;
  float a;
  if (gi < n && gj < n && vmode == VAL_LINEAR) {
    a = (float)((double)D[e] + (gi == gj ? lambda : 0.0));
  } else if (gi < n && gj < n) {  // the same value as the Gram epilogue
    const int64_t dmax = etab_len - 1;
    const int32_t dc = (int32_t)min((int64_t)max(D[e], 0), dmax);
    double ev = (vmode == VAL_EXP && dmax / EXP_LO + 1 <= EXP_HI_MAX)
                    ? etab[(int64_t)(dc / EXP_LO) * EXP_LO] * etab[dc % EXP_LO]
                    : etab[dc];
    if (Ec) ev *= Ec[e];
    a = (gi == gj) ? (float)(1.0 + lambda) : (float)ev;
  } else {
    a = (gi == gj) ? 1.0f : 0.0f;
  }
  A[e] = a;
}

void launch_expand_tiles(const int32_t *D, const double *etab, int64_t etab_len, double lambda,
                         int vmode, const double *Ec, const TileLayout &L, float *A,
                         hipStream_t s) {
  const int64_t total = L.elems();
  hipLaunchKernelGGL(k_expand_tiles, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, D,
                     etab, etab_len, lambda, L.n, L.nb, total, vmode, Ec, A);
}

// IBS kernel (Algorithm 5, IBS branch): the alleles two patients share
// identical by state, over the 2m alleles of a patient.  With the
// thermometer encoding h(g) = ([g >= 1], [g >= 2]) of each genotype,
// ||h(a) - h(b)||^2 = |a - b| for a, b in {0, 1, 2}, so the squared distance
// of the encoded rows is d = sum_k |g_ik - g_jk| (exact, through the same
// INT8 Gram), the shared alleles are 2m - d, and K_ij = (2m - d) / (2m):
// tab[d] for d = 0 .. 2m (larger d cannot occur; they read 0).
__global__ void k_ibs_table(double *tab, int64_t len, int64_t m) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d < len) tab[d] = d <= 2 * m ? (double)(2 * m - d) / (double)(2 * m) : 0.0;
}

void launch_ibs_table(double *tab, int64_t len, int64_t m, hipStream_t s) {
  hipLaunchKernelGGL(k_ibs_table, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, tab, len,
                     m);
}

// Thermometer encoding of genotype rows: H[i, c] = [g_ic >= 1] for c < m and
// H[i, half + c] = [g_ic >= 2], half = m rounded up to 16; the columns
// m .. half-1 and half+m .. 2 half-1 are zero.  16 genotypes per thread.
__global__ void k_ibs_encode(const int8_t *__restrict__ G, int64_t rows, int64_t m, int64_t ldg,
                             int8_t *__restrict__ H, int64_t ldh, int64_t half) {
  const int64_t per_row = half / 16;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * per_row) return;
  const int64_t i = e / per_row, c0 = (e % per_row) * 16;
  const uint8_t *g = (const uint8_t *)G + i * ldg + c0;
  uint32_t w[4];
  *(v4i *)w = *(const v4i *)g;  // in bounds: ldg is a multiple of 16 and >= m
  uint32_t h1[4], h2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t valid = m - c0 - 4 * q;
    uint32_t x = w[q];
    if (valid <= 0) x = 0;
    else if (valid < 4) x &= (1u << (8 * valid)) - 1u;
    // per byte b in {0, 1, 2}: [b >= 1] = (b | b >> 1) & 1, [b >= 2] = (b >> 1) & 1
    h1[q] = (x | (x >> 1)) & 0x01010101u;
    h2[q] = (x >> 1) & 0x01010101u;
  }
  int8_t *o = H + i * ldh + c0;
  *(v4i *)o = *(const v4i *)h1;
  *(v4i *)(o + half) = *(const v4i *)h2;
}

void launch_ibs_encode(const int8_t *G, int64_t rows, int64_t m, int64_t ldg, int8_t *H,
                       int64_t ldh, hipStream_t s) {
  const int64_t half = (m + 15) / 16 * 16;
  const int64_t tot = rows * (half / 16);
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_ibs_encode, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, G, rows,
                     m, ldg, H, ldh, half);
}

// Confounder factors of the Gaussian kernel (the Build subsection adds the
// squared distances of real-valued covariates to the genotype distances
// before the exponential): Ec_ij = exp(-gamma dc_ij), dc_ij = sum_k (c_ik -
// c_jk)^2 by its definition in FP64, over the packed lower tiles (1 on
// padding rows and columns).  One 64 x 64 block per workgroup, the 64 + 64
// confounder rows it needs staged in LDS.
constexpr int CONF_QMAX = 32;

__global__ __launch_bounds__(256) void k_conf_factor(const double *__restrict__ C, int64_t n,
                                                     int64_t q, int64_t ldc, double gamma, int nb,
                                                     double *__restrict__ Ec) {
  __shared__ double ci[64][CONF_QMAX + 1], cj[64][CONF_QMAX + 1];
  const int sb = nb / 64, nsub = sb * sb;
  const int64_t t = blockIdx.x / nsub;
  const int sub = (int)(blockIdx.x % nsub), si = sub / sb, sj = sub % sb;
  int I, J;
  tri_decode(t, I, J);
  const int64_t i0 = (int64_t)I * nb + si * 64, j0 = (int64_t)J * nb + sj * 64;
  for (int e = threadIdx.x; e < 64 * (int)q; e += 256) {
    const int r = e / (int)q, k = e % (int)q;
    ci[r][k] = (i0 + r < n) ? C[(i0 + r) * ldc + k] : 0.0;
    cj[r][k] = (j0 + r < n) ? C[(j0 + r) * ldc + k] : 0.0;
  }
  __syncthreads();
  double *out = Ec + t * (int64_t)nb * nb + (int64_t)(si * 64) * nb + sj * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    double v = 1.0;
    if (i0 + r < n && j0 + c < n) {
      double dc = 0.0;
      for (int k = 0; k < (int)q; ++k) {
        const double x = ci[r][k] - cj[c][k];
        dc = fma(x, x, dc);
      }
      v = exp(-gamma * dc);
    }
    out[(int64_t)r * nb + c] = v;
  }
}

void launch_conf_factor(const double *C, int64_t n, int64_t q, int64_t ldc, double gamma,
                        const TileLayout &L, double *Ec, hipStream_t s) {
  const int sb = L.nb / 64;
  hipLaunchKernelGGL(k_conf_factor, dim3((unsigned)(L.ntiles() * sb * sb)), dim3(256), 0, s, C, L.n,
                     q, ldc, gamma, L.nb, Ec);
}

// The same factors between test rows (Ct, rows x q) and training rows (C):
// Et[i, j] = exp(-gamma sum_k (ct_ik - c_jk)^2) for j < n, 1 for the padding
// columns n .. cols-1; row-major with leading dimension lde.
__global__ __launch_bounds__(256) void k_conf_factor_cross(const double *__restrict__ Ct,
                                                           int64_t rows, int64_t ldct,
                                                           const double *__restrict__ C, int64_t n,
                                                           int64_t q, int64_t ldc, double gamma,
                                                           int64_t cols, double *__restrict__ Et,
                                                           int64_t lde) {
  __shared__ double ci[64][CONF_QMAX + 1], cj[64][CONF_QMAX + 1];
  const int64_t ncb = (cols + 63) / 64;
  const int64_t i0 = (int64_t)(blockIdx.x / ncb) * 64, j0 = (int64_t)(blockIdx.x % ncb) * 64;
  for (int e = threadIdx.x; e < 64 * (int)q; e += 256) {
    const int r = e / (int)q, k = e % (int)q;
    ci[r][k] = (i0 + r < rows) ? Ct[(i0 + r) * ldct + k] : 0.0;
    cj[r][k] = (j0 + r < n) ? C[(j0 + r) * ldc + k] : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    if (i0 + r >= rows || j0 + c >= cols) continue;
    double v = 1.0;
    if (j0 + c < n) {
      double dc = 0.0;
      for (int k = 0; k < (int)q; ++k) {
        const double x = ci[r][k] - cj[c][k];
        dc = fma(x, x, dc);
      }
      v = exp(-gamma * dc);
    }
    Et[(i0 + r) * lde + j0 + c] = v;
  }
}

void launch_conf_factor_cross(const double *Ct, int64_t rows, int64_t ldct, const double *C,
                              int64_t n, int64_t q, int64_t ldc, double gamma, int64_t cols,
                              double *Et, int64_t lde, hipStream_t s) {
  const int64_t blocks = ((rows + 63) / 64) * ((cols + 63) / 64);
  hipLaunchKernelGGL(k_conf_factor_cross, dim3((unsigned)blocks), dim3(256), 0, s, Ct, rows, ldct,
                     C, n, q, ldc, gamma, cols, Et, lde);
}

// Cross distances for Predict (Algorithm 4's Build(gamma, T, G)):
// Dt[i, j] = n^T_i + n^G_j - 2 <t_i, g_j> for i < rows, j < cols_padded
// (0 for the padding columns j >= n), or the inner product <t_i, g_j>
// itself for the linear kernel.  Row-major with leading dimension ldd.
template <class S>
__global__ __launch_bounds__(S::THREADS) void k_cross_gram(const int8_t *__restrict__ T, int64_t rows,
                                                    const int32_t *__restrict__ nrm_t,
                                                    const int8_t *__restrict__ G, int64_t n,
                                                    int64_t m, int64_t ldt, int64_t ldg,
                                                    const int32_t *__restrict__ nrm_g,
                                                    int64_t cols, int64_t nbc,
                                                    int32_t *__restrict__ Dt, int64_t ldd,
                                                    int linear) {
  constexpr int BM = S::kBM, BN = S::kBN;
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  const int64_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t bi = bid / nbc, bj = bid % nbc;
  const int64_t row0 = bi * BM, col0 = bj * BN;
  const int arows = (int)max((int64_t)0, min((int64_t)BM, rows - row0));
  const int brows = (int)max((int64_t)0, min((int64_t)BN, n - col0));
  OpI8::acc_t acc[S::WTM][S::WTN];
  zero_acc(acc);
  if (arows > 0 && brows > 0)
    gemm_nt_stream<OpI8, S>(
        ContigSrc<OpI8>{(const uint8_t *)T + row0 * ldt, (const uint8_t *)G + col0 * ldg, OpI8{}},
        ldt, arows, ldg, brows, m, acc, lds);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int tm = 0; tm < S::WTM; ++tm)
#pragma unroll
    for (int tn = 0; tn < S::WTN; ++tn)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t gi = row0 + S::row(wave, tm, i, lane);
        const int64_t gj = col0 + S::col(wave, tn, lane);
        if (gi < rows && gj < cols)
          Dt[gi * ldd + gj] = (gj >= n)  ? 0
                              : linear   ? acc[tm][tn][i]
                                         : nrm_t[gi] + nrm_g[gj] - 2 * acc[tm][tn][i];
      }
}

void launch_cross_gram(const int8_t *T, int64_t nt_rows, const int32_t *nrm_t, const int8_t *G,
                       int64_t n, int64_t m, int64_t ldt, int64_t ldg, const int32_t *nrm_g,
                       int64_t cols_padded, int32_t *Dt, int64_t ldd, bool linear,
                       hipStream_t s) {
  constexpr int BM = GramShape::kBM, BN = GramShape::kBN;
  const int64_t nbr = (nt_rows + BM - 1) / BM, nbc = (cols_padded + BN - 1) / BN;
  build_kernel_attrs();
  hipLaunchKernelGGL((k_cross_gram<GramShape>), dim3((unsigned)(nbr * nbc)),
                     dim3(GramShape::THREADS), GramShape::LDS_BYTES, s, T,
                     nt_rows, nrm_t, G, n, m, ldt, ldg, nrm_g, cols_padded, nbc, Dt, ldd,
                     linear ? 1 : 0);
}

// Diagnostics: gather a rectangular block of a tile-packed symmetric matrix.
template <typename T>
__global__ void k_copy_tiles(const T *__restrict__ src, int nb, int64_t i0, int64_t j0,
                             int64_t rows, int64_t cols, int lower_only, T *__restrict__ dst,
                             int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = i0 + e / cols, j = j0 + e % cols;
  T v;
  if (lower_only && j > i) {
    v = (T)0;
  } else {
    const int64_t a = i >= j ? i : j, b = i >= j ? j : i;  // symmetric: read lower
    const int64_t I = a / nb, J = b / nb;
    int64_t r = a % nb, c = b % nb;
    if (I == J && !lower_only) {  // diagonal tiles are stored in full
      r = i % nb;
      c = j % nb;
    }
    v = src[(I * (I + 1) / 2 + J) * (int64_t)nb * nb + r * nb + c];
  }
  dst[(e / cols) * ld + e % cols] = v;
}

void launch_copy_tiles_i32(const int32_t *D, const TileLayout &L, int64_t i0, int64_t j0,
                           int64_t rows, int64_t cols, int32_t *dst, int64_t ld, hipStream_t s) {
  const int64_t tot = rows * cols;
  hipLaunchKernelGGL(k_copy_tiles<int32_t>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     D, L.nb, i0, j0, rows, cols, 0, dst, ld);
}

void launch_copy_tiles_f32(const float *A, const TileLayout &L, int64_t i0, int64_t j0,
                           int64_t rows, int64_t cols, bool lower_only, float *dst, int64_t ld,
                           hipStream_t s) {
  const int64_t tot = rows * cols;
  hipLaunchKernelGGL(k_copy_tiles<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, A,
                     L.nb, i0, j0, rows, cols, lower_only ? 1 : 0, dst, ld);
}

}  // namespace krr

namespace krr {

// Transpose of an int8 matrix: At[c, i] = A[i, c] for i < rows, c < cols, and
// zeros in the padding columns rows .. ldt-1 of At.  64 x 64 blocks through LDS.
__global__ __launch_bounds__(256) void k_transpose_i8(const int8_t *__restrict__ A, int64_t rows,
                                                      int64_t cols, int64_t lda,
                                                      int8_t *__restrict__ At, int64_t ldt) {
  __shared__ int8_t t[64][65];
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e / 64, c = e % 64;
    t[r][c] = (r0 + r < rows && c0 + c < cols) ? A[(r0 + r) * lda + c0 + c] : (int8_t)0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int c = e / 64, r = e % 64;  // output row c0 + c, column r0 + r
    if (c0 + c < cols && r0 + r < ldt) At[(c0 + c) * ldt + r0 + r] = t[r][c];
  }
}

void launch_transpose_i8(const int8_t *A, int64_t rows, int64_t cols, int64_t lda, int8_t *At,
                         int64_t ldt, hipStream_t s) {
  const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((ldt + 63) / 64));
  hipLaunchKernelGGL(k_transpose_i8, grid, dim3(256), 0, s, A, rows, cols, lda, At, ldt);
}

// B = A^T Y for an int8 matrix A (rows x cols, row-major) and FP64 Y (rows x
// r, column-major, ldy): B[a, c] = sum_i A[i, a] Y[i, c] in FP64 with the sum
// over i in order; B column-major (ldb).  A workgroup owns 64 columns a and
// 16 columns c (four per thread); the rows are staged 64 at a time (the A
// block and the Y block in LDS).  The products of small integers with FP64
// values are exact, so only the additions round.
__global__ __launch_bounds__(256) void k_int8_t_times_f64(const int8_t *__restrict__ A,
                                                          int64_t rows, int64_t cols, int64_t lda,
                                                          const double *__restrict__ Y, int r,
                                                          int64_t ldy, double *__restrict__ B,
                                                          int64_t ldb) {
  __shared__ int8_t as[64][64 + 4];
  __shared__ double ys[64][17];
  const int64_t a0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 16;
  const int al = threadIdx.x % 64, cg = threadIdx.x / 64;  // column a0 + al, c0 + 4 cg .. +3
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = 0; i0 < rows; i0 += 64) {
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int ii = e / 64, aa = e % 64;
      as[ii][aa] = (i0 + ii < rows && a0 + aa < cols) ? A[(i0 + ii) * lda + a0 + aa] : (int8_t)0;
    }
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int cc = e / 64, ii = e % 64;
      ys[ii][cc] = (i0 + ii < rows && c0 + cc < r) ? Y[(int64_t)(c0 + cc) * ldy + i0 + ii] : 0.0;
    }
    __syncthreads();
    for (int ii = 0; ii < 64; ++ii) {
      const double g = (double)as[ii][al];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = fma(g, ys[ii][4 * cg + q], acc[q]);
    }
    __syncthreads();
  }
  if (a0 + al < cols)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (c0 + 4 * cg + q < r) B[(int64_t)(c0 + 4 * cg + q) * ldb + a0 + al] = acc[q];
}

void launch_int8_t_times_f64(const int8_t *A, int64_t rows, int64_t cols, int64_t lda,
                             const double *Y, int r, int64_t ldy, double *B, int64_t ldb,
                             hipStream_t s) {
  const dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((r + 15) / 16));
  hipLaunchKernelGGL(k_int8_t_times_f64, grid, dim3(256), 0, s, A, rows, cols, lda, Y, r, ldy, B,
                     ldb);
}

// Dynamic-LDS limits of the Gram kernels (above the 64 KB default), set once
// per process before their first launch; the context's creation calls it, so
// that it never runs inside a stream capture.
void build_kernel_attrs() {
  static bool done = false;
  if (done) return;
  done = true;
  (void)hipFuncSetAttribute((const void *)k_gram_tiles<GramShape>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GramShape::LDS_BYTES);
  (void)hipFuncSetAttribute((const void *)k_gram_tiles_batched<GramShape>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GramShape::LDS_BYTES);
  (void)hipFuncSetAttribute((const void *)k_cross_gram<GramShape>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, GramShape::LDS_BYTES);
}

}  // namespace krr
