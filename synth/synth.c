/*
 * Seeded synthetic genotype generator.
 *
 * Test and benchmark infrastructure only: it produces inputs, and holds none
 * of the kernel-ridge-regression arithmetic.  Both the GPU library's tests and
 * the CPU oracle draw their inputs from here, so that a row block can be
 * regenerated anywhere from (seed, stream, row index) alone.
 *
 * Random numbers come from Philox4x32-10, the counter-based generator
 * published by Salmon, Moraes, Dror and Shaw ("Parallel random numbers: as
 * easy as 1, 2, 3", SC'11), written here from that definition: ten rounds of
 * two 32x32->64 multiplies with the published multipliers, a Feistel-style
 * swap, and a Weyl-sequence key schedule.
 *
 * Counter layout for genotype (row i, SNP pair q = j/2):
 *     ctr = (i_lo, i_hi, q, stream),  key = (seed_lo, seed_hi)
 * The four output words u0..u3 give SNP 2q from (u0, u1) and SNP 2q+1 from
 * (u2, u3):  g = [u_a < t_j] + [u_b < t_j], t_j = floor(p_j * 2^32), i.e. a
 * Binomial(2, p_j) draw with p_j the minor-allele frequency of SNP j.
 */
#include <stdint.h>
#include <stddef.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static inline void philox4x32_10(const uint32_t in[4], uint32_t k0, uint32_t k1,
                                 uint32_t out[4]) {
  uint32_t x0 = in[0], x1 = in[1], x2 = in[2], x3 = in[3];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Raw Philox block, exported so tests can compare with the published
 * known-answer vectors. */
void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                         uint32_t out[4]) {
  philox4x32_10(ctr, key[0], key[1], out);
}

/*
 * Genotypes for rows [row0, row0 + rows) and all m SNPs, written row-major
 * into out (leading dimension ld >= m).  thresh[j] = floor(p_j * 2^32).
 */
void synth_genotypes(int8_t *out, int64_t rows, int64_t m, int64_t ld,
                     int64_t row0, const uint32_t *thresh, uint64_t seed,
                     uint32_t stream) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    const uint64_t gi = (uint64_t)(row0 + r);
    int8_t *dst = out + r * ld;
    uint32_t ctr[4], u[4];
    ctr[0] = (uint32_t)gi;
    ctr[1] = (uint32_t)(gi >> 32);
    ctr[3] = stream;
    for (int64_t q = 0; 2 * q < m; ++q) {
      ctr[2] = (uint32_t)q;
      philox4x32_10(ctr, k0, k1, u);
      const int64_t j = 2 * q;
      uint32_t t = thresh[j];
      dst[j] = (int8_t)((u[0] < t) + (u[1] < t));
      if (j + 1 < m) {
        t = thresh[j + 1];
        dst[j + 1] = (int8_t)((u[2] < t) + (u[3] < t));
      }
    }
  }
}

/*
 * Linkage-disequilibrium blocks, applied in place after synth_genotypes:
 * for each block b starting at SNP founder[b] and covering len SNPs, SNP
 * founder[b]+s (s >= 1) copies the founder's genotype per patient, except
 * that with probability 'resample' (as a 2^-32-scaled threshold) it is
 * redrawn from Binomial(2, p_founder).  Uses stream 'stream' so the draws are
 * independent of the base genotypes.
 */
void synth_ld_blocks(int8_t *out, int64_t rows, int64_t m, int64_t ld,
                     int64_t row0, const int64_t *founder, int64_t nblocks,
                     int64_t len, const uint32_t *thresh, uint32_t resample,
                     uint64_t seed, uint32_t stream) {
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    const uint64_t gi = (uint64_t)(row0 + r);
    int8_t *dst = out + r * ld;
    uint32_t ctr[4], u[4];
    ctr[0] = (uint32_t)gi;
    ctr[1] = (uint32_t)(gi >> 32);
    ctr[3] = stream;
    for (int64_t b = 0; b < nblocks; ++b) {
      const int64_t f = founder[b];
      const uint32_t t = thresh[f];
      for (int64_t s = 1; s < len && f + s < m; ++s) {
        ctr[2] = (uint32_t)(b * len + s);
        philox4x32_10(ctr, k0, k1, u);
        if (u[0] < resample)
          dst[f + s] = (int8_t)((u[1] < t) + (u[2] < t));
        else
          dst[f + s] = dst[f];
      }
    }
  }
}
