// Host-side declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/krr.h"

namespace krr {

// Lower-triangle tile layout of an np x np matrix (np = nt * nb).
struct TileLayout {
  int nb = 512;
  int nt = 0;
  int64_t n = 0;   // logical size
  int64_t np = 0;  // padded size
  int64_t ntiles() const { return (int64_t)nt * (nt + 1) / 2; }
  int64_t tile_elems() const { return (int64_t)nb * nb; }
  int64_t elems() const { return ntiles() * tile_elems(); }
  static int64_t tri(int64_t I, int64_t J) { return I * (I + 1) / 2 + J; }
};

// One instance of a batched solve (device table): the factor, the FP32
// right-hand sides of the sweeps (row-major np x r), and what the FP64
// residual reads and writes.
struct SolveJob {
  const float *Lst, *Linv;
  float *B, *Z, *X;
  int nt;
  const int32_t *D;
  const double *etab;
  int64_t etab_len;
  double gamma;
  int wshift;           // residual_exp_shift(gamma, etab_len)
  int64_t np;
  const double *Xd;     // FP64 iterate
  double *part;         // residual_split * np * r partial products
  int64_t rb0;          // first residual row block of this instance
};

// ---- build.hip ----
// One instance of a batched Build: its inputs, outputs and the first
// workgroup of each batched launch that belongs to it.
struct BuildJob {
  const int8_t *G;
  int64_t n, np, ldg;
  int32_t *nrm;
  int32_t *flag;        // genotype check of this instance
  double *etab;         // exp(-gamma d), d = 0 .. etab_len-1
  int64_t etab_len;
  double gamma, lambda;
  int32_t *D;
  float *A;
  double *part;         // per-sub-block sums of squares
  double *tnorm;        // per-tile Frobenius norms
  int64_t ntiles;
  int64_t row0;         // first row-norm workgroup
  int64_t block0;       // first Gram workgroup
};
// Batched Build launches over jobs[0 .. njobs-1] (device memory); rows and
// blocks are the totals over the batch (last job's row0 + np, block0 + its
// blocks).
void launch_row_norms_batched(const BuildJob *jobs, int njobs, int64_t rows, int64_t m,
                              hipStream_t s);
void launch_exp_tables_batched(const BuildJob *jobs, int njobs, int64_t max_len, hipStream_t s);
int64_t gram_blocks(const TileLayout &L);  // Gram workgroups of one instance
void launch_gram_tiles_batched(const BuildJob *jobs, int njobs, int64_t blocks, int64_t m, int nb,
                               hipStream_t s);
int gram_parts(int nb);  // partial sums per tile
void launch_tile_norms_batched(const BuildJob *jobs, int njobs, int64_t max_ntiles, int nb,
                               hipStream_t s);
void launch_exp_table(double *tab, int64_t len, double gamma, hipStream_t s);
void launch_row_norms(const int8_t *G, int64_t n, int64_t rows_padded, int64_t m, int64_t ldg,
                      int32_t *nrm, int32_t *flag, hipStream_t s);
// How a stored integer becomes the kernel value: the exponential of the
// distance (Gaussian), a table of the distance (IBS), the integer itself
// (linear kernel: the stored integer is the inner product, not a distance).
enum { VAL_EXP = 0, VAL_TABLE = 1, VAL_LINEAR = 2 };
// vmode: VAL_*; Ec: FP64 confounder factors in the packed tile layout, or null.
// Gs (or null): G in slab-major order (launch_slab_major), read instead of G.
void launch_gram_tiles(const int8_t *G, int64_t m, int64_t ldg, const int32_t *nrm,
                       const double *etab, int64_t etab_len, double lambda, const TileLayout &L,
                       int32_t *D, float *A, double *tnorm_part, int vmode,
                       const double *Ec, const int8_t *Gs, hipStream_t s);
// Gs[(s np + r) 64 + b] = G[r, 64 s + b] (zero past m and for rows n .. np-1):
// np * ceil(m / 64) * 64 bytes.
// The slab-major copy of G with its row norms (nrm zeroed first, then summed
// in) and the genotype check (flag |= 1 on a byte above 2), one pass.
void launch_slab_major_norms(const int8_t *G, int64_t n, int64_t np, int64_t m, int64_t ldg,
                             int8_t *Gs, int32_t *nrm, int32_t *flag, hipStream_t s);
void launch_slab_major(const int8_t *G, int64_t n, int64_t np, int64_t m, int64_t ldg,
                       int8_t *Gs, hipStream_t s);
void launch_tile_norms(const double *part, int parts, int64_t ntiles, double *tnorm, hipStream_t s);
void launch_expand_tiles(const int32_t *D, const double *etab, int64_t etab_len, double lambda,
                         int vmode, const double *Ec, const TileLayout &L, float *A,
                         hipStream_t s);
// At (cols x ldt) = A^T with zero padding columns; B = A^T Y in FP64 (A int8
// rows x cols row-major, Y and B column-major).
void launch_transpose_i8(const int8_t *A, int64_t rows, int64_t cols, int64_t lda, int8_t *At,
                         int64_t ldt, hipStream_t s);
void launch_int8_t_times_f64(const int8_t *A, int64_t rows, int64_t cols, int64_t lda,
                             const double *Y, int r, int64_t ldy, double *B, int64_t ldb,
                             hipStream_t s);
// IBS kernel: table (2m - d) / (2m), and the thermometer encoding of genotype
// rows (H: rows x ldh int8, ldh >= 2 * round_up(m, 16), a multiple of 16).
void launch_ibs_table(double *tab, int64_t len, int64_t m, hipStream_t s);
void launch_ibs_encode(const int8_t *G, int64_t rows, int64_t m, int64_t ldg, int8_t *H,
                       int64_t ldh, hipStream_t s);
// Confounder factors exp(-gamma ||c_i - c_j||^2) (FP64, q <= 32): packed lower
// tiles of the training set, and test rows x training columns.
constexpr int KRR_CONF_QMAX = 32;
void launch_conf_factor(const double *C, int64_t n, int64_t q, int64_t ldc, double gamma,
                        const TileLayout &L, double *Ec, hipStream_t s);
void launch_conf_factor_cross(const double *Ct, int64_t rows, int64_t ldct, const double *C,
                              int64_t n, int64_t q, int64_t ldc, double gamma, int64_t cols,
                              double *Et, int64_t lde, hipStream_t s);
void launch_cross_gram(const int8_t *T, int64_t nt_rows, const int32_t *nrm_t, const int8_t *G,
                       int64_t n, int64_t m, int64_t ldt, int64_t ldg, const int32_t *nrm_g,
                       int64_t cols_padded, int32_t *Dt, int64_t ldd, bool linear,
                       hipStream_t s);
void launch_copy_tiles_i32(const int32_t *D, const TileLayout &L, int64_t i0, int64_t j0,
                           int64_t rows, int64_t cols, int32_t *dst, int64_t ld, hipStream_t s);
void launch_copy_tiles_f32(const float *A, const TileLayout &L, int64_t i0, int64_t j0,
                           int64_t rows, int64_t cols, bool lower_only, float *dst, int64_t ld,
                           hipStream_t s);

// ---- factor.hip ----
struct UpdatePolicy {
  int mode;          // KRR_POLICY_*
  int allow16, allow8;  // precisions the rule may choose
  int have16 = 0;       // FP16 operands reachable (the rule, or FP8 promoted one level)
  int high_panels;
  int fixed_prec;
  int rule;          // KRR_RULE_* (ADAPTIVE)
  double thr;        // eps * ||A||_F / NT
  const uint8_t *fmap = nullptr;  // FIXED_MAP: precision per (panel, tile), device
  const uint8_t *pcap = nullptr;  // lowest precision allowed per panel (promotion), or null
  const double *tnorm = nullptr;  // per-tile ||A_IJ||_F of the build (KRR_RULE_TILE / BOTH)
};
// Operand copies of one panel (tiles k+1 .. nt-1 of block column k).  Two
// are kept so that panel k+1 can be produced while panel k is still read.
struct PanelBuf {
  float *P32 = nullptr;       // FP32 L_ik
  _Float16 *P16 = nullptr;    // FP16 copies
  uint8_t *P8 = nullptr;      // FP8 E4M3 copies of 2^pexp8 L_ik
  float *pnorm = nullptr;     // ||L_ik||_F
  int *pexp8 = nullptr;       // FP8 scale exponents
};
constexpr int KRR_MAX_GROUP = 8;  // panels per grouped trailing update
// Workspace for the factorization, sized for nt tiles of nb.
struct FactorWork {
  // diagonal tiles, FP64 (or FP32 under the plain policy)
  double *W64 = nullptr;     // nb x nb: the tile being factored
  double *WL64 = nullptr;    // nt x nb x nb: the factors L_kk
  double *Dinv64 = nullptr;  // nt x (nb/64) inverses of their 64 x 64 diagonal blocks
  double *Winv64 = nullptr;  // inv_chunk x nb x nb: tile inverses, a chunk at a time
  double *Tmp64 = nullptr;   // inv_chunk x nb x nb / 2
  int inv_chunk = 16;
  PanelBuf pb[2 * KRR_MAX_GROUP];  // two groups of panel operand copies
  double *pnorm_part = nullptr;  // (nt-1) * parts (max((nb/64)^2, nb/16))
  float *pmax_part = nullptr;    // (nt-1) * parts
  int32_t *flag = nullptr;       // breakdown column + 1 (0 = none)
  unsigned long long *counts = nullptr;  // [3] updates per precision
  // split-K load of a diagonal tile: per-chunk 64 x 64 partial products
  // (KRR_MAX_GROUP chunks x (nb/64)(nb/64+1)/2 blocks)
  float *lpart = nullptr;
  double *WX64 = nullptr;  // nb x nb: the next row tile's panel while the steps form it
};
// Updates of a diagonal tile left to its factorization: P[q] points at tile
// k of panel buffer q; pmap_at[q] is the precision-map entry to mark FP32.
struct DiagUpdate {
  const float *P[KRR_MAX_GROUP];
  int64_t pmap_at[KRR_MAX_GROUP];
  uint8_t *pmap;
  int npan;
};
constexpr int KRR_SLOTS = 2 * KRR_MAX_GROUP;  // panel buffers of a workspace
// One instance of a lockstep batched factorization (device table): its
// factor storage, its workspace (diagonal tiles in the factorization's
// type, FP64 or FP32) and panel buffers, and its precision threshold.
struct FactorJob {
  float *Lst, *Linv;
  void *W, *WL, *Dinv, *Winv, *Tmp;
  float *P32[KRR_SLOTS];
  _Float16 *P16[KRR_SLOTS];
  uint8_t *P8[KRR_SLOTS];
  float *pnorm[KRR_SLOTS];
  int *pexp8[KRR_SLOTS];
  double *pnorm_part;
  float *pmax_part;
  int32_t *flag;
  uint8_t *pmap;
  int64_t ntiles;
  double thr;  // eps * ||A||_F / nt
  const double *tnorm;  // the build's tile norms (tile precision rule)
  int nt;
};
// The single-stream tile Cholesky (substitution TRSM, grouped updates of g
// panels, panel k in buffer ((k / g) % 2) g + k % g) of njobs instances in
// lockstep: every POTRF step, TRSM, conversion and update is one launch for
// all instances that have that step; the panel is solved as a product with
// the tile inverse, formed right after the tile's factor (L_kk and its
// inverse stored as krr_factor stores them).  nts: host copy of the tile
// counts; pol.thr is taken per instance from the table.
void launch_factor_lockstep(const FactorJob *jobs, const int *nts, int njobs, int nb, int g,
                            const UpdatePolicy &pol, bool fp64, bool need16, bool need8,
                            bool scale8, hipStream_t s);
// Diagonal tile k: L_kk = chol(A_kk - sum_q P_q P_q^T) into the work's
// factor store (tile k), with the inverses of its 64 x 64 diagonal blocks.
// Linv_k (or null): also L_kk in FP32 into Akk and block rows 0 .. nb/64-2 of
// inv(L_kk) in FP32 into Linv_k, formed in the same steps (the last block
// row by launch_tile_inverse_last_row); needs at least two tiles of the
// work's inverse chunk buffer.
// The next row tile's panel formed in the same steps (RowPanel::A non-null):
// P = A inv(L_kk)^T for A = A_k+1,k (FP32, row-major nb x nb), by the steps'
// extra workgroups (right-looking, block column by block column, in the
// work's WX64 tile), into P32 (FP32) with the per-64x64-block sums of squares
// and maxima (parts slots a tile) the panel conversion reads; `wait`, if not
// null, is waited for between the tile's load and its steps (A ready).
struct RowPanel {
  const float *A = nullptr;
  float *P32 = nullptr;
  double *pnorm_part = nullptr;
  float *pmax_part = nullptr;
  int parts = 0;
  hipEvent_t wait = nullptr;
};
void launch_potrf_tile(float *Akk, int k, const TileLayout &L, bool fp64, FactorWork &w,
                       const DiagUpdate &du, float *Linv_k, hipStream_t s,
                       const RowPanel &row = RowPanel{});
int trsm_parts(int nb);  // partial-norm slots of a panel tile
void launch_tile_inverse_last_row(float *Linv_k, int k, const TileLayout &L, bool fp64,
                                  FactorWork &w, hipStream_t s);
// L_kk into the factor storage and inv(L_kk), FP32, for the diagonal tiles
// k_lo .. k_hi-1 (factored before).
void launch_tile_inverses(float *Lst, float *Linv, int k_lo, int k_hi, const TileLayout &L,
                          bool fp64, FactorWork &w, hipStream_t s);
// Coupling tiles C_p = inv(L_k+1,k+1) L_k+1,k inv(L_kk) of the tile pairs
// (k, k+1) = (2p, 2p+1), p < nt / 2, for the paired sweeps; Tmp, C: nt / 2 tiles.
void launch_sweep_coupling(const float *Lst, const float *Linv, const TileLayout &L, float *Tmp,
                           float *C, hipStream_t s);
// Coupling tiles Q = inv(P1) M inv(P0) of the tile quads (4q .. 4q+3), q < nt / 4,
// for sweeps that take four tiles a step (P0, P1 its pairs, M the 2 x 2 tiles
// between them; Cpair from launch_sweep_coupling); Tmp, Q: 4 (nt / 4) tiles,
// Q's four tiles of quad q at 4q (00, 01, 10, 11).
void launch_quad_coupling(const float *Lst, const float *Linv, const float *Cpair,
                          const TileLayout &L, float *Tmp, float *Q, hipStream_t s);
// P_i = A_ik inv(L_kk)^T for the tiles i = k+1+t, t_lo <= t < t_hi: by
// substitution with the factor of tile k (no inverse needed), or as a product
// with inv(L_kk) (launch_tile_inverses first).
void launch_trsm_subst(const float *Astore, int k, const TileLayout &L, bool fp64, FactorWork &w,
                       const PanelBuf &pb, int t_lo, int t_hi, hipStream_t s);
void launch_trsm_gemm(const float *Astore, const float *Linv_k, int k, const TileLayout &L,
                      FactorWork &w, const PanelBuf &pb, int t_lo, int t_hi, hipStream_t s);
// pol (or null): write only the operand copies some update of each tile will
// read under this policy (the tile norms, their extremes and the rule);
// otherwise every copy need16 / need8 asks for.
void launch_convert_panel(float *Astore, int k, const TileLayout &L, FactorWork &w, bool scale8,
                          const PanelBuf &pb, bool need16, bool need8, const UpdatePolicy *pol,
                          hipStream_t s);
// Trailing update of the tiles (i, j), jlo <= j <= jhi, j <= i, by the npan
// consecutive panels k0 .. k0+npan-1 whose operand copies are *pbs[q].
void launch_update(float *Astore, int k0, int npan, int jlo, int jhi, const TileLayout &L,
                   const UpdatePolicy &pol, FactorWork &w, const PanelBuf *const *pbs,
                   uint8_t *pmap, int which, hipStream_t s);
enum { UPD_ALL = 0, UPD_DIAG = 1, UPD_OFFDIAG = 2 };  // tiles launch_update covers
// counts[p] += number of entries of pmap equal to p (p = 0, 1, 2)
void launch_count_pmap(const uint8_t *pmap, int64_t n, unsigned long long *counts,
                       hipStream_t s);

void launch_encode_fp8(const float *x, int64_t n, uint8_t *out, hipStream_t s);

// ---- solve.hip ----
// Internal right-hand sides are row-major np x r.
// Right-hand sides of these two: FP32 column-major np x r (column stride
// np).  C: the coupling tiles of launch_sweep_coupling (tiles taken in
// pairs), or null (one tile per step).
// sp (or null): a second stream and nev events; with it each quad step's
// panel is split in two launches, the next quad's tiles on s and the rest
// on s2, so that the rest overlaps the next quad's diagonal step (s2 is
// joined back into s before the sweep returns).
struct SweepSplit {
  hipStream_t s2;
  hipEvent_t *ev;
  int nev;
};
void launch_fwd_sweep(const float *Astore, const float *Linv, const float *C, const float *Q,
                      const TileLayout &L, int r, float *B, float *Z, hipStream_t s,
                      const SweepSplit *sp = nullptr);
void launch_bwd_sweep(const float *Astore, const float *Linv, const float *C, const float *Q,
                      const TileLayout &L, int r, float *Z, float *X, hipStream_t s,
                      const SweepSplit *sp = nullptr);
// the sweeps take the tiles in quads when given Q (tile 256, wide panels)
bool sweep_quads_supported(int nb);
// R = Y - (K + lambda I) X in FP64; part: residual_split(L) * np * r doubles
// of workspace for the partial products.
int residual_split(const TileLayout &L);
// the same for the lockstep batch (at most residual_split)
int residual_split_batched(const TileLayout &L);
// vmode: VAL_* (VAL_EXP factors the exponential when gamma allows); Ec: FP64
// confounder factors (packed like D) multiplied into every entry, or null.
// nsplit: tile-column ranges summed in fixed order (clamped to 1 .. nt); part
// holds nsplit * np * r doubles.
void launch_residual(const int32_t *D, const double *etab, int64_t etab_len, double gamma,
                     int vmode, const double *Ec, double lambda, const TileLayout &L, int r,
                     const double *X, const double *Y, double *R, double *part, int nsplit,
                     hipStream_t s);
// The same residual with every stored tile of D read once (each tile's two
// products into slots of their own, summed in fixed order): part holds
// residual_once_bytes(L, r) bytes (NT * np * r doubles).
int64_t residual_once_bytes(const TileLayout &L, int r);
void launch_residual_once(const int32_t *D, const double *etab, int64_t etab_len, double gamma,
                          int vmode, const double *Ec, double lambda, const TileLayout &L, int r,
                          const double *X, const double *Y, double *R, double *part,
                          hipStream_t s);
// Batched (lockstep over a table of instances, tile counts up to ntmax):
// both sweeps, L Z = B then L^T X = Z.
void launch_sweeps_batched(const SolveJob *jobs, int njobs, int ntmax, int nb, int r,
                           hipStream_t s);
// log2 of the residual's exp factoring width for (gamma, 4m + 1), or -1
int residual_exp_shift(double gamma, int64_t etab_len);
// partial products of every instance (rblocks = total np / 64; fact when every
// instance has wshift >= 0), then per instance R = Y - sum part - lambda X
void launch_residual_batched(const SolveJob *jobs, int njobs, int64_t rblocks, bool fact, int nb,
                             int r, hipStream_t s);
void launch_residual_sum(const double *part, int nsplit, const TileLayout &L, int r,
                         double lambda, const double *X, const double *Y, double *R,
                         hipStream_t s);
void launch_colmajor_to_rows(const double *src, int64_t n, int64_t ld, int r, int64_t np,
                             double *dst, hipStream_t s);
void launch_rows_to_colmajor(const double *src, int64_t n, int r, double *dst, int64_t ld,
                             hipStream_t s);
void launch_f64_to_f32(const double *src, int64_t count, float *dst, hipStream_t s);
// row-major FP64 np x r -> column-major FP32, and dst += alpha src back
void launch_rows_f64_to_cols_f32(const double *src, int64_t np, int r, float *dst,
                                 hipStream_t s);
void launch_cols_f32_axpy_rows_f64(const float *src, int64_t np, int r, double alpha, double *dst,
                                   hipStream_t s);
void launch_axpy_f32_to_f64(const float *src, int64_t count, double alpha, double *dst,
                            hipStream_t s);
// Column dot products / squared norms of row-major n x r FP64 matrices into
// out[0 .. r); ws: col_dots_workspace(r) doubles.
int col_dots_workspace(int r);
void launch_col_norms(const double *A, int64_t n, int r, double *out, double *ws, hipStream_t s);
void launch_col_dots(const double *A, const double *B, int64_t n, int r, double *out, double *ws,
                     hipStream_t s);
// Preconditioned conjugate gradients on the columns of row-major count / r x r
// matrices: x += alpha p, res -= alpha A p from nq = -A p, alpha = rho / (p . A p)
// with pnq = p . nq; then p = z + (rho_new / rho_old) p (p = z when rho_old is null).
void launch_pcg_step(double *x, double *res, const double *p, const double *nq, const double *rho,
                     const double *pnq, int64_t count, int r, hipStream_t s);
void launch_pcg_dir(double *p, const double *z, const double *rho_new, const double *rho_old,
                    int64_t count, int r, hipStream_t s);
// Et (or null): factors multiplied into the entries, row-major like Dt;
// linear: Dt holds inner products, which are the values.
void launch_predict_apply(const int32_t *Dt, int64_t rows, int64_t cols, int64_t ldd,
                          const double *etab, int64_t etab_len, const double *X, int r, double *P,
                          int64_t ldp, const double *Et, bool linear, hipStream_t s);
void launch_fill_f64(double *p, int64_t count, double v, hipStream_t s);
void launch_fill_i32(int32_t *p, int64_t count, int32_t v, hipStream_t s);
void launch_fill_u8(uint8_t *p, int64_t count, uint8_t v, hipStream_t s);

// Dynamic-LDS attributes of the kernels that need more than 64 KB, set once
// per process (the context's creation calls them, outside any capture).
void build_kernel_attrs();
void factor_kernel_attrs();
void solve_kernel_attrs();

}  // namespace krr
