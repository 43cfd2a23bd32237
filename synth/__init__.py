"""Seeded synthetic GWAS inputs: genotypes, minor-allele frequencies, phenotypes.

Test and benchmark infrastructure shared by the oracle's tests and the GPU
library's tests and benchmark.  It holds none of the kernel-ridge-regression
arithmetic: it only draws inputs.

The real cohorts the paper uses (UK BioBank 305,880 x 43,333; msprime
300K x 40K) are not available, so these seeded synthetic matrices stand in for
them, with the shapes of the benchmark workloads:

* genotypes G[i, j] in {0, 1, 2}: Binomial(2, p_j) per SNP j, drawn with the
  counter-based Philox4x32-10 generator in ``synth.c`` (row-addressable: any
  row block can be regenerated from (seed, stream, row));
* minor-allele frequencies p_j from numpy's PCG64 seeded with the workload
  seed (uniform or clipped Beta);
* phenotypes: sums of epistatic pair products beta_k * G[:, a_k] * G[:, b_k]
  and additive terms theta_l * G[:, c_l], plus Gaussian noise, each column then
  standardised (mean 0, sd 1, ddof = 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile synth.c into libsynth.so with gcc (OpenMP over rows)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.synth_philox4x32_10.argtypes = [P, P, P]
        lib.synth_philox4x32_10.restype = None
        lib.synth_genotypes.argtypes = [P, I64, I64, I64, I64, P, ctypes.c_uint64, ctypes.c_uint32]
        lib.synth_genotypes.restype = None
        lib.synth_ld_blocks.argtypes = [P, I64, I64, I64, I64, P, I64, I64, P,
                                        ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32]
        lib.synth_ld_blocks.restype = None
        _lib = lib
    return _lib


def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (for known-answer tests)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    _load().synth_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def thresholds(p: np.ndarray) -> np.ndarray:
    """Per-SNP uint32 thresholds floor(p * 2^32) for Binomial(2, p) draws."""
    return np.floor(np.asarray(p, np.float64) * 2.0 ** 32).astype(np.uint32)


def maf_uniform(m: int, lo: float, hi: float, seed: int) -> np.ndarray:
    return np.random.default_rng([seed, 1]).uniform(lo, hi, m)


def maf_beta(m: int, a: float, b: float, lo: float, hi: float, seed: int) -> np.ndarray:
    return np.clip(np.random.default_rng([seed, 1]).beta(a, b, m), lo, hi)


def genotypes(n: int, m: int, p: np.ndarray, seed: int, stream: int = 0, row0: int = 0,
              out: np.ndarray | None = None, ld_blocks: tuple | None = None) -> np.ndarray:
    """int8 genotype rows [row0, row0+n) x m SNPs, row-major (SNP-contiguous).

    ``ld_blocks = (founders, length, resample_prob)`` adds linkage blocks.
    """
    if out is None:
        out = np.empty((n, m), np.int8)
    assert out.dtype == np.int8 and out.shape[0] >= n and out.shape[1] >= m
    assert out.strides[1] == 1
    t = np.ascontiguousarray(thresholds(p))
    lib = _load()
    lib.synth_genotypes(out.ctypes.data, n, m, out.strides[0], row0, t.ctypes.data,
                        ctypes.c_uint64(seed), ctypes.c_uint32(stream))
    if ld_blocks is not None:
        founders, length, prob = ld_blocks
        f = np.ascontiguousarray(founders, dtype=np.int64)
        lib.synth_ld_blocks(out.ctypes.data, n, m, out.strides[0], row0, f.ctypes.data,
                            len(f), length, t.ctypes.data,
                            ctypes.c_uint32(int(prob * 2.0 ** 32)),
                            ctypes.c_uint64(seed), ctypes.c_uint32(stream + 1))
    return out


def ld_founders(m: int, frac: float, length: int, seed: int) -> np.ndarray:
    """Start SNPs of non-overlapping, aligned linkage blocks covering ~frac of SNPs."""
    nblocks = int(round(frac * m / length))
    slots = m // length
    rng = np.random.default_rng([seed, 3])
    return np.sort(rng.choice(slots, size=nblocks, replace=False)) * length


def confounders(n: int, q: int, seed: int, sd: float, row0: int = 0) -> np.ndarray:
    """Real-valued covariates (n x q, float64, row-major) standing in for the
    confounders of a cohort (principal components, age, sex and the like):
    column 0 a binary indicator, the others N(0, sd^2), one seeded stream
    per row so that any row block can be regenerated."""
    out = np.empty((n, q), np.float64)
    for i in range(n):
        rng = np.random.default_rng([seed, 4, row0 + i])
        v = rng.standard_normal(q) * sd
        v[0] = sd * float(rng.integers(0, 2))
        out[i] = v
    return out


def phenotypes(G: np.ndarray, r: int, n_pairs: int, n_add: int, seed: int,
               h2: float | None = None, noise_sd: float | None = None) -> np.ndarray:
    """Phenotype matrix Y (n x r, float64, column-major) with epistatic signal.

    Column c: g = sum_k beta_k G[:, a_k] G[:, b_k] + sum_l theta_l G[:, c_l], with
    distinct random SNPs and beta, theta ~ N(0, 1); noise is N(0, noise_sd^2) when
    ``noise_sd`` is given, else has variance Var(g) (1 - h2) / h2.  Each column is
    then standardised (mean 0, sd 1, ddof = 0).
    """
    n, m = G.shape
    rng = np.random.default_rng([seed, 2])
    Y = np.empty((n, r), np.float64, order="F")
    for c in range(r):
        snps = rng.choice(m, size=2 * n_pairs + n_add, replace=False)
        beta = rng.standard_normal(n_pairs)
        theta = rng.standard_normal(n_add)
        cols = G[:, snps].astype(np.float64)
        g = (cols[:, 0:2 * n_pairs:2] * cols[:, 1:2 * n_pairs:2]) @ beta
        if n_add:
            g += cols[:, 2 * n_pairs:] @ theta
        if noise_sd is not None:
            sd = noise_sd
        else:
            var = g.var()
            sd = np.sqrt(var * (1.0 - h2) / h2) if var > 0 else 1.0
        y = g + sd * rng.standard_normal(n)
        y -= y.mean()
        s = y.std()
        Y[:, c] = y / (s if s > 0 else 1.0)
    return Y


@dataclass
class Workload:
    """One synthetic KRR problem: sizes, hyperparameters and generator seeds."""
    name: str
    n: int
    m: int
    r: int
    gamma: float
    lam: float
    seed: int
    maf: tuple = ("uniform", 0.05, 0.5)
    pheno: dict = field(default_factory=dict)
    n_test: int = 0
    ld: tuple | None = None  # (fraction, block length, resample probability)

    def maf_vector(self) -> np.ndarray:
        kind = self.maf[0]
        if kind == "uniform":
            return maf_uniform(self.m, self.maf[1], self.maf[2], self.seed)
        if kind == "beta":
            return maf_beta(self.m, *self.maf[1:], seed=self.seed)
        raise ValueError(kind)

    def ld_spec(self):
        if self.ld is None:
            return None
        frac, length, prob = self.ld
        return (ld_founders(self.m, frac, length, self.seed), length, prob)

    def genotypes(self, rows: int | None = None, row0: int = 0) -> np.ndarray:
        """Training rows (row0 .. row0+rows) of the genotype stream."""
        rows = self.n if rows is None else rows
        return genotypes(rows, self.m, self.maf_vector(), self.seed, 0, row0,
                         ld_blocks=self.ld_spec())

    def test_genotypes(self) -> np.ndarray:
        """Test patients: the rows that follow the n training rows in the same stream."""
        return genotypes(self.n_test, self.m, self.maf_vector(), self.seed, 0, self.n,
                         ld_blocks=self.ld_spec())

    def phenotypes(self, G: np.ndarray) -> np.ndarray:
        return phenotypes(G, self.r, seed=self.seed, **self.pheno)


_BASE_SEED = 240901712 * 10

# The five workload shapes of the benchmark description.  The first is the
# small case the oracle finishes in seconds; the second is the throughput
# workload on one GPU.  gamma = 1/M on raw integer squared distances.
WORKLOADS = {
    "small": Workload("small", 2048, 4096, 1, 1.0 / 4096, 0.1, _BASE_SEED + 0,
                      pheno=dict(n_pairs=20, n_add=0, noise_sd=0.5)),
    "single": Workload("single", 32768, 65536, 16, 1.0 / 65536, 0.1, _BASE_SEED + 1,
                       pheno=dict(n_pairs=50, n_add=10, h2=0.5)),
    "large": Workload("large", 131072, 262144, 64, 1.0 / 262144, 0.05, _BASE_SEED + 2,
                      maf=("uniform", 0.01, 0.5), ld=(0.05, 32, 0.1),
                      pheno=dict(n_pairs=50, n_add=10, h2=0.5)),
    "trainpredict": Workload("trainpredict", 200000, 100000, 128, 1.0 / 100000, 0.1,
                             _BASE_SEED + 4, maf=("beta", 0.5, 2.0, 0.01, 0.5),
                             pheno=dict(n_pairs=50, n_add=10, h2=0.5), n_test=20000),
}


def batched_workloads(count: int = 48, m: int = 16384, r: int = 8, seed: int = _BASE_SEED + 3,
                      n_lo: int = 1024, n_hi: int = 16384, step: int = 256):
    """Batch of independent KRR instances with uneven N and differing (gamma, lambda).

    N_b ~ U{n_lo, n_lo + step, ..., n_hi}; gamma cycles over {0.5, 1, 2}/M and lambda
    over {1e-3, 1e-2, 1e-1, 1}, so every (gamma, lambda) pair occurs count/12 times.
    Instance b takes its genotype rows from one shared stream at a row offset.
    """
    rng = np.random.default_rng([seed, 4])
    ns = rng.integers(n_lo // step, n_hi // step + 1, size=count) * step
    gam = [0.5 / m, 1.0 / m, 2.0 / m]
    lam = [1e-3, 1e-2, 1e-1, 1.0]
    out, row0 = [], 0
    for b in range(count):
        w = Workload("batch%d" % b, int(ns[b]), m, r, gam[b % 3], lam[(b // 3) % 4], seed,
                     pheno=dict(n_pairs=50, n_add=10, h2=0.5))
        out.append((w, row0))
        row0 += int(ns[b])
    return out
