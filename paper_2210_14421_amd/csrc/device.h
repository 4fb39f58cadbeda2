// Device-side data of a context and the launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace efe {

// Geometry and 1-D tables needed by most kernels (passed by value).
struct Geom {
  int nc[3];
  int64_t nn[3];
  int p, P, nloc;
  int64_t cstride;   // elements between stored cell blocks: nloc^2 rounded up to 8 (16-byte aligned blocks)
  int qc, qe;
  int64_t n_nodes;
};

// Offsets of the 1-D tables inside the device table buffer (doubles).
struct TabOff {
  int Bc, dBc, Be, dBe;     // [n][P]
  int xqc, wqc, xqe, wqe;   // [n]
  int G1c, G1e;             // [n][NP]: B[i][a] B[i][a'] per unordered pair
  int Kr, Mr;               // [P][P] reference-cell stiffness / mass (cell edge h: 2/h Kr, h/2 Mr)
  int xb[3];                // per axis: the nc[d] + 1 cell boundaries
  int pair;                 // [P][P] pair index (as doubles)
  int total;
};

// Partial reorthogonalisation state of the Lanczos columns: three rows of omega
// estimates [3][ld][ncol] (rows by Lanczos index modulo 3, ld = kmax + 2), the
// running ||T|| estimate and the forced-pass flag per column.
struct ProState {
  double *om = nullptr;
  double *anorm = nullptr;
  int *force = nullptr;
  int ld = 0;
};

struct DevData {
  Geom g;
  TabOff to;
  double *tab = nullptr;          // 1-D tables
  uint8_t *is_enr = nullptr;      // n_cells
  int64_t *q_off = nullptr;       // n_cells + 1
  int *cells_ord = nullptr, *cells_enr = nullptr;   // ordinary / enrichment cell ids
  int n_ord = 0, n_enr = 0;
  int *colour_cells = nullptr;    // cells grouped by colour
  int *cell_slot = nullptr;       // n_cells: storage slot of the cell block (colour-major order)
  int colour_off[9] = {0};
  // cells of each colour by class (sum-factorised products): colour c's ordinary cells are
  // sf_ord[sf_off[2c] .. sf_off[2c+2]), its enrichment cells sf_enr[sf_off[2c+1] .. sf_off[2c+3])
  int *sf_ord = nullptr, *sf_enr = nullptr;
  int sf_off[18] = {0};
  double *D = nullptr, *Dm12 = nullptr;   // lumped mass, D^-1/2 (0 on boundary)
  double *vstatic = nullptr;      // n_quad
  double *occ = nullptr;          // norb
  // enrichment
  int ne = 0, nk = 0, nt = 0;     // enrichment functions, kept directions, T-cells
  int max_tnu = 0;                // most enrichment functions nonzero on one T-cell
  int64_t nr = 0;                 // union rows
  int *tcell = nullptr, *tnu_off = nullptr, *tnu = nullptr;
  int *tslot_of_cell = nullptr;   // n_cells, -1 if not a T-cell
  int64_t *tne_off = nullptr;     // per slot, N^E values
  double *NE = nullptr;
  int64_t *tpart_off = nullptr;   // per slot: offset into the coupling partials (nloc * nnu)
  int64_t *thee_off = nullptr;    // per slot: offset into H^ee partials (nnu^2)
  int16_t *tpos = nullptr;        // [slot][ne]: local index of nu in the slot's list, -1
  int64_t *urow_node = nullptr;
  int *urow_cnt = nullptr, *urow_pair = nullptr;
  double *S = nullptr;            // ne x nk
  double *C = nullptr;            // nr x ne: orthogonalisation coefficients c on the union rows
  int *node_urow = nullptr;       // n_nodes: union row of the node, -1
  int *ta_off = nullptr, *ta_nu = nullptr;   // per slot: enrichment functions with an atomic part there
  int64_t *tna_off = nullptr;     // per slot: offset of its atomic values
  double *NA = nullptr;           // s_nu N^A_nu(q) at the points of those slots
  int max_ta = 0;                 // most atomic functions on one T-cell
  double *Kce = nullptr;          // nr x ne
  double *Kee = nullptr;          // ne x ne
  // Poisson
  double *K1[3] = {nullptr, nullptr, nullptr}, *M1[3] = {nullptr, nullptr, nullptr};
  double *fdmV[3] = {nullptr, nullptr, nullptr}, *fdmL[3] = {nullptr, nullptr, nullptr};
  double *fdmVT[3] = {nullptr, nullptr, nullptr};   // transposes of fdmV (rows of the back transform)
  double *gbnd = nullptr, *lift = nullptr;
};

// Kernel launchers (stream-ordered, no synchronisation).
namespace k {

constexpr int kDotBlocksMax = 1024;   // partial blocks of the column reductions
constexpr int kCoupleScratch = 520;  // n_k x ncolr blocks: workgroup partials and first-level sums of Y_E
constexpr int kAlphaParts = 4;       // partials of x^H Hbar x per (column, cell): one per wave of a column half

void zero(double *p, int64_t n, hipStream_t s);
void copy_rows(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t nrows, int ncolr, hipStream_t s);
void axpby(const double *x, const double *y, double a, double b, double *out, int64_t n, hipStream_t s);

// rebuild of the cell blocks: mode 0 = Hamiltonian, 1..3 = position operator x/y/z
void rebuild_cells(const DevData &d, int mode, const double *rho, const double *phi, const double *efield, int fdir,
                   int xc, void *cells, int dtype, double *vq, hipStream_t s);
void coupling_partials(const DevData &d, const double *vq, double *part, double *hee_part, hipStream_t s);
// G = Hbar^ce on the union rows, in FP64 (G), or in FP32 (G32, when G is null)
void coupling_gather(const DevData &d, const double *part, int kinetic, double *G, float *G32, hipStream_t s);
// scratch: hee_scratch_size(d) doubles
int64_t hee_scratch_size(const DevData &d);
void hee_reduce(const DevData &d, const double *hee_part, int kinetic, double *Hee_raw, double *Hbar_ee,
                double *scratch, hipStream_t s);

// Hbar X
// raises the dynamic LDS limit of the cell-product kernels for cells of nloc nodes; 0 on success
int cell_apply_init(int nloc);
// apart (FP64 blocks only, else ignored): per column and cell, the sum of X Y over the nodes
// the cell's colour reaches last (Y the stored sum of all cell products), in kAlphaParts
// partials at apart[(col * n_cells + cell slot) * kAlphaParts + part] (cell slots in colour order)
void cell_apply(const DevData &d, const void *cells, int dtype, const double *X, double *Y, int ncolr, int64_t ldr,
                hipStream_t s, const int *any = nullptr, int variant = 0, double *apart = nullptr);
// the same with FP32 Y (ldf floats per row, a multiple of 4) and X in the reduced-precision
// copy: FP32 for FP32 and split BF16 blocks, BF16 for BF16 blocks
void cell_apply_f(const DevData &d, const void *cells, int dtype, const void *X, float *Y, int ncolr, int64_t ldf,
                  hipStream_t s, const int *any = nullptr, int variant = 0);
// BF16 products (16x16x32 BF16 MFMA, FP32 accumulation): blocks of planes (1: BF16,
// 2: hi/lo split) BF16 planes of nloc rows padded to 8 elements; raises the LDS limit
int cell_bf16_init(int nloc);
int64_t bf16_block_elems(const Geom &g, int planes);
void cell_apply_bf16(const DevData &d, const uint16_t *cells, int planes, const double *X, double *Y, int ncolr,
                     int64_t ldr, hipStream_t s, const int *any = nullptr, int variant = 0);
void cell_apply_bf16_f(const DevData &d, const uint16_t *cells, int planes, const void *X, int x_bf16, float *Y,
                       int ncolr, int64_t ldf, hipStream_t s, const int *any = nullptr, int variant = 0);
// variants of the BF16 products: 0 eight waves, 1 twelve waves per workgroup; 2 and 3 the
// same with the block rows loaded through registers; 4 and 5 with three stages of the
// block rows in LDS (2 to 5: one BF16 plane only)
int cell_bf16_variant_count(int nloc, int planes);
// pipeline variants of the cell products that fit the LDS for cells of nloc nodes and
// blocks of esz bytes (all give the same bits; variant 0 is the default), and their names
int cell_variant_count(int nloc, size_t esz);
// sixteen-wave variants of the FP32 block products (ids written to out[<= 3]; none for
// FP64 blocks or cells of more than 256 nodes)
int cell_wide_variants(int nloc, size_t esz, int *out);
void cell_variant_name(int v, char *out, int len);
// narrow-tile variants (64 columns per workgroup for FP64 and FP32 blocks, 32 for FP32 blocks)
// worth trying for ncolr real columns (degree <= 5): their ids in out[], their number returned
int cell_narrow_variants(int nloc, int ncolr, size_t esz, int *out);
// sum-factorised cell products (FP64, no stored blocks): Y = sum_c P_c^T Hbar_c P_c X from the
// potential at the quadrature points (vq) and, with kinetic, the kinetic term
bool sf_supported(const Geom &g);
int sf_init(const Geom &g);
void sf_apply(const DevData &d, const double *vq, int kinetic, const double *X, double *Y, int ncolr, int64_t ldr,
              hipStream_t s, const int *any = nullptr);
// aE (optional): the enrichment terms of x^H Hbar x per (function, column), nk x ncolr
void couple_apply(const DevData &d, const double *G, const double *Hee, const double *X, double *Y,
                  int ncolr, int64_t ldr, double *scratch, hipStream_t s, const int *any = nullptr,
                  double *aE = nullptr);
// the FP32 coupling (G in FP32, FP32 MFMA) on FP64 rows X and Y
void couple_apply_g32(const DevData &d, const float *G, const double *Hee, const double *X, double *Y, int ncolr,
                      int64_t ldr, double *scratch, hipStream_t s, const int *any = nullptr);
// FP32 coupling products (FP32 MFMA; G and Y in FP32, Y with ldf floats per row); X: the
// FP32 copy (ldf floats per row), or, when X64 is given, the packed FP64 rows
void couple_apply_f(const DevData &d, const float *G, const double *Hee, const float *X, const double *X64,
                    float *Y, int ncolr, int64_t ldf, double *scratch, hipStream_t s, const int *any = nullptr);

// density and Poisson
// workspace of the density: U holds the folded union rows (n_R x ncolr), part
// the per-pass partial sums on the enrichment cells (density_part_size doubles)
struct DenWork {
  double *U = nullptr, *part = nullptr;
};
bool density_folded_ok(const DevData &d);
int64_t density_part_size(const DevData &d, int ncolr);
void psiE(const DevData &d, const double *X, int ncolr, int64_t ldr, double *psiE, hipStream_t s);
// raises the dynamic LDS limit of the density kernels; 0 on success
int density_init(const Geom &g);
void density(const DevData &d, const double *X, int ncol, int64_t ldr, const double *psiE, double *rho,
             const DenWork &w, hipStream_t s);
void poisson_rhs(const DevData &d, const double *rho, double *dvec, double *rhs, hipStream_t s, int lift = 1);
// adjoint pieces
void cross_density(const DevData &d, const double *Z, int npair, const double *psiE, double w, double *out,
                   const DenWork &work, hipStream_t s);
void adj_potential(const DevData &d, const double *phibar, const double *rho, const double *u, double tau, int xc,
                   const double mubar[3], double a, const double *gin, double *out, hipStream_t s);
void axpy_cols(double *out, const double *Y, const double *sc, double s0, int64_t nrows, int ncol, hipStream_t s);
void interleave(const double *a, const double *b, double *Z, int64_t nrows, int ncol, hipStream_t s);
void stiffness_apply(const DevData &d, const double *x, double *y, double *t1, double *t2, hipStream_t s,
                     const int *skip = nullptr);
void fdm_apply(const DevData &d, const double *r, double *z, double *t1, double *t2, hipStream_t s,
               const int *skip = nullptr);
// device-side PCG pieces (all skipped while *skip != 0)
void axpby_dev(const double *x, const double *y, double a, const double *b, double *out, int64_t n, const int *skip,
               hipStream_t s);
void pcg_update(double *x, double *r, const double *p, const double *q, const double *alpha, int64_t n,
                const int *skip, hipStream_t s);
void pcg_scalar(int op, double *S, double tol2, int *done, hipStream_t s);
void set_scalar(double *p, double v, hipStream_t s);
void set_boundary(const DevData &d, double *phi, hipStream_t s);
// partial dot products: out[blk] partials; returns number of blocks used
int dot_partials(const double *x, const double *y, int64_t n, double *part, hipStream_t s);
void reduce_partials(const double *part, int nblk, int nval, double *out, hipStream_t s);
void dipole_partials(const DevData &d, const double *rho, double *part, int *nblk, hipStream_t s);

// absorption spectrum (Sec. 3.2): S[nw], alpha[ndir][nw][2] (may be null) from traces mu[ndir][nt1][3]
// P[i] = |int exp(-t^2/tau) mu_dir''(t) exp(-i omega_i t) dt|^2 (mu: device [nt1][3], nt1 >= 3)
void power_spectrum(const double *mu, int dir, int64_t nt1, double dt, double tau, const double *omega, int64_t nw,
                    double *P, hipStream_t st);
void spectrum(const double *mu, const int *dirs, int ndir, int64_t nt1, double dt, double tau, int kind,
              double kappa, double t0, double s, const double *omega, int64_t nw, double *S, double *alpha,
              hipStream_t st);

// Lanczos vectors (unnormalised basis: slot 0 = q0, slot l >= 1 = qb + (l - 1) * bs)
int lz_dots(const double *q0, const double *qb, int64_t bs, int nq, const double *w, int64_t nrows, int ncol,
            const int *mask, const int *any, int with_norm, double *part, hipStream_t s);
// in place on w; sh (optional): reduced-precision copy of the result (FP32, or BF16 with
// sh_bf16), shld elements per row
int lz_update(const double *q0, const double *qb, int64_t bs, int nq, const double *coef, const double *gw, double *w,
              int64_t nrows, int ncol, const int *mask, const int *any, double *part, hipStream_t s,
              int zero_masked = 0, void *sh = nullptr, int64_t shld = 0, int sh_bf16 = 0);
// reduced-precision products: the dots with an FP32 product block (ldf floats per row), and
// the first update reading it (src) into the FP64 slot w with a reduced-precision copy of the
// result in sh (FP32, or BF16 with sh_bf16; ldf elements per row)
int lz_dots_f(const double *q0, const double *qb, int64_t bs, int nq, const float *w, int64_t ldf, int64_t nrows,
              int ncol, const int *mask, const int *any, int with_norm, double *part, hipStream_t s);
int lz_update_from(const double *q0, const double *qb, int64_t bs, int nq, const double *coef, const double *gw,
                   const float *src, int64_t ldf, double *w, void *sh, int sh_bf16, int64_t nrows, int ncol,
                   const int *mask, const int *any, double *part, hipStream_t s, int zero_masked);
// packed FP64 block (ncolr values per row) <-> FP32 block of ldf floats per row (pad columns zero)
void to_f32(const double *X, int64_t nrows, int ncolr, float *Xf, int64_t ldf, hipStream_t s);
// packed FP64 block -> reduced-precision copy (FP32, or BF16 with bf16) of ldf elements per row
void to_shadow(const double *X, int64_t nrows, int ncolr, void *Xs, int64_t ldf, int bf16, hipStream_t s);
void from_f32(const float *Xf, int64_t ldf, int64_t nrows, int ncolr, double *X, hipStream_t s);
// nq_dev (optional): device count that bounds nq (the largest k of the columns)
void lz_combine(const double *q0, const double *qb, int64_t bs, int nq, const double *coef, double *out,
                int64_t nrows, int ncol, hipStream_t s, const int *nq_dev = nullptr);
void lz_kmax(const int *kused, int ncol, int *kmaxu, hipStream_t s);
void lz_init(const double *h0, int ncol, double *beta0, double *sig, int *active, int *kused, const ProState &pro,
             hipStream_t s);
// first: the first slot of the dot pass the coefficients come from (0: all slots)
void lz_coef1(const double *h, const double *sig, int j, int first, int ncol, const int *active, double *alpha_j,
              double *coef, double *gsc, double *msc, hipStream_t s);
// three-term step of iteration j from the dot with slot j - 1 and the known beta_{j-1}
void lz_coef3(const double *h, const double *sig, const double *beta, int j, int ncol, const int *active,
              double *alpha_j, double *coef, double *gsc, double *msc, hipStream_t s);
constexpr int kAlphaLvl = 16;   // first-level sums of x^H Hbar x per real column (lz_alpha_coef3 workspace)
// the three-term step of iteration j with x^H Hbar x of slot j - 1 from the products' shares:
// apart[col][part] (nparts cell partials per real column) and aE[k][col] (nk enrichment terms),
// each summed in a fixed order (lvl: kAlphaLvl x 2 ncol doubles of workspace)
void lz_alpha_coef3(const double *apart, int nparts, const double *aE, int nk, double *lvl, const double *sig,
                    const double *beta, int j, int ncol, const int *active, const int *any, double *alpha_j,
                    double *coef, double *gsc, double *msc, hipStream_t s);
// partial reorthogonalisation decision after the local pass of iteration j (sets need, any);
// rel: the update pass was not scaled to a unit input, so the cancellation test divides by
// the input's norm (the second entry of nrm1)
void lz_pro(const double *nrm1, const double *msc, const double *alpha, const double *beta, int j, int ncol,
            const int *active, const ProState &pro, int *need, int *any, hipStream_t s, int rel = 0);
void lz_decide(const double *nrm1, int ncol, const int *active, const double *gsc, int *need, int *any,
               hipStream_t s);
void lz_coef2(const double *h2, const double *nrm1, const double *sig, int j, int ncol, const int *need, double *coef,
              double *gsc, double *msc, hipStream_t s);
void lz_beta(const double *nrm1, const double *nrm2, const int *need, const int *active, const double *msc, int j,
             int ncol, double *beta_j, double *sig, hipStream_t s);
// any = OR of the active flags of ncol columns
void lz_any(const int *active, int ncol, int *any, hipStream_t s);
void lz_comb_coef(const double *u, const double *sig, const double *beta0, const int *kused, int kmax, int nl,
                  int ncol, double *coef, hipStream_t s);
// combination coefficients [m][kmax][ncol] (complex) of a finished Lanczos at the times taus[0..m), m <= 16
void tridiag_coef(const double *alpha, const double *beta, const int *kused, int ncol, int kmax, const double *taus,
                  int m, const double *beta0, const double *sig, double *coef, hipStream_t s);
void tridiag_exp(const double *alpha, const double *beta, int j, int ncol, int kmax, double tau,
                 const double *beta0, const int *kforce, double tol, int *active, int *kused, double *err,
                 double *u, hipStream_t s);
}  // namespace k
}  // namespace efe
