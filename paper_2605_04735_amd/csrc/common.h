// Internal declarations shared by the HIP kernels and the C-ABI driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace topo {

// ---------------------------------------------------------------- device scalars
// Float64 scalars of a running solve live in one small device array so that
// consecutive kernels hand them over without a host round trip.
enum Scal {
  S_RZ = 0,     // r^T z of the current CG iterate
  S_ALPHA,      // CG step length
  S_BETA,       // CG direction update factor
  S_RR,         // ||r||^2 over free DOFs (recursive residual)
  S_TOL2,       // stop when S_RR <= S_TOL2
  S_PQ,         // p^T K p
  S_NORM2,      // ||f - K u||^2 of the outer residual
  S_SCALE,      // 1/||f - K u||: scaling of the inner right-hand side
  S_C,          // compliance f^T u
  S_ES,         // sum_e E_e u_e^T k0 u_e
  S_TMP,
  S_RZ0,        // r^T z of the partial-sum set of parity 0 / 1 (batched CG)
  S_RZ1,
  S_RP,         // bfloat16 directions: r^T p_old of the current iterate (see CGP_RP)
  S_AH,         // grouped x update: step length of the direction in slot j, S_AH + j
  S_COUNT = S_AH + 4 + 4
};
enum Flag {
  F_DONE = 0,   // inner CG finished (converged, broke down or non-finite)
  F_STATUS,     // 0 ok, 1 breakdown (p^T K p <= 0), 2 non-finite
  F_ITERS,      // inner CG iterations of the current inner solve
  F_BADX,       // bit 0: some x outside [0,1]; bit 1: some x non-finite
  F_CAP,        // the inner CG stops (done) after this many iterations
  F_BADG,       // some sensitivity handed to the OC update is non-finite
  F_SLOT0,      // direction slot of the first product of the current inner solve
  F_COUNT = 8
};

constexpr int MAXB = 8192;         // capacity of the per-block partial-sum array
constexpr int RED_THREADS = 256;

// ---------------------------------------------------------------- OC update
// Textbook optimality-criteria bisection: lam in [0, OC_L2_0], stop when
// (l2 - l1) / (l1 + l2) <= OC_TOL, at most OC_MAX_STEPS midpoints.
constexpr double OC_L2_0 = 1e9;
constexpr double OC_TOL = 1e-3;
constexpr int OC_MAX_STEPS = 200;
constexpr int OC_THREADS = 256;
constexpr int OC_MAXB = 1024;      // blocks of an OC launch
// bracket state, two copies (alternate launches read one and write the other)
enum OcState { OC_L1 = 0, OC_L2, OC_LAM, OC_DONE, OC_STEPS, OC_STATE = 8 };
// OC scratch (doubles): partials [2][OC_MAXB], state [2][OC_STATE], output [8]
constexpr int OC_STATE_OFS = 2 * OC_MAXB;
constexpr int OC_OUT_OFS = OC_STATE_OFS + 2 * OC_STATE;
constexpr int OC_SCRATCH = OC_OUT_OFS + 8;

// Element tile of the matrix-free product: TEX x TEY elements per z layer, one
// thread each; the tile owns the TNX x TNY nodes whose all adjacent elements
// lie in it, and marches up a z range of node planes.  Its node plane is
// TPX x TPY.
#ifndef TOPO_TEX
#define TOPO_TEX 32
#define TOPO_TEY 8
#endif
constexpr int TEX = TOPO_TEX, TEY = TOPO_TEY;
constexpr int TNX = TEX - 1, TNY = TEY - 1;
constexpr int TPX = TEX + 1, TPY = TEY + 1;
constexpr int MV_THREADS = TEX * TEY;
static_assert(MV_THREADS == 256 || MV_THREADS == 512, "one 256- or 512-thread block per tile");
// block-count targets below are for 256-thread blocks; scaled by this
constexpr int MV_BLOCK_SCALE = MV_THREADS / 256;
static_assert(TEX == 16 || TEX == 32 || TEX == 64, "x rows of 16, 32 or 64 lanes");
static_assert(TPX * TPY <= 2 * MV_THREADS, "a node plane is staged in two slots per thread");

enum MvMode { MV_APPLY = 0, MV_CG = 1, MV_RESID = 2 };

// Tile of the matrix-core (MFMA) float32 product: ME x ME elements per z
// layer, MN x MN owned nodes (see k_mfma.hip).
constexpr int ME = 16, MN = ME - 1;
constexpr int MF_THREADS = 256;  // its blocks: 4 waves of 4 element rows

// Unit-modulus coefficients of the factored hex8 stiffness (see k_matvec.hip),
// already multiplied by h/32.
template <typename T>
struct Coef {
  T L2, M4, M2, L2_3, M2_3, B9;
};

template <typename T>
struct MvArgs {
  int nelx, nely, nelz, kz;
  const T *E;            // [nel] moduli
  const T *in;           // APPLY/RESID: u; CG: z
  const T *pold;         // CG: previous search direction
  T *pout;               // CG: new search direction (owned nodes)
  T *out;                // APPLY: y; CG: q = K p; RESID: r = f - K u
  const double *f;       // RESID: load vector
  const uint8_t *mask;   // [nn] bit c set = DOF c fixed
  double *part;          // [nblocks] partial sums (CG: p^T q; RESID: ||r||^2)
  const double *scal;    // CG: reads S_BETA
  const int *flags;      // CG: early exit when flags[F_DONE]
  Coef<T> k;
  const void *mA;        // matrix-core float32 product: the A operand (2 x 64 x 16 bytes)
  float mscale;          //   and the element scale h mu / 72 (times E_e)
  // CG: with zfuse, `in` is the residual r and the product forms z = D r from
  // the Jacobi inverse diagonal (otherwise `in` is the z the update stored)
  const T *dinv;         // [nn]
  int zfuse;
};

// Direction slots of the inner CG: the product of slot s reads p[s] as the
// previous direction and writes p[(s + 1) % np]; its partial sums alternate
// with s & 1.  Without grouping every update advances x by alpha p.  With
// grouped x the updates keep each step length and advance x once every np
// iterations by the np steps together (the update of slot np - 2, when all np
// directions are still in their slots): x += alpha p moves 36 bytes per node,
// the grouped form 12 + 24 / np on average.
constexpr int CG_NP_MAX = 4;
enum XUpdate { XU_EACH = 0, XU_SKIP = 1, XU_FLUSH2 = 2, XU_FLUSH4 = 3 };

// One design of a batched inner CG solve (device resident).
template <typename T>
struct CgDesc {
  int nelx, nely, nelz, kz;
  int tx, ty;           // product tiles along x and y (blocks: tx * ty * tz)
  int nb_mv, nb_up;     // blocks of this design in the product / update kernels
  int zbf16;           // float32 CG: z stored in bfloat16 (2 bytes per component)
  int zfuse;           // the product forms z = D r (1) or reads the z the update stored (0)
  int np;              // direction slots: 2 (0 reads as 2) or 4
  int xgroup;          // x advanced once per np iterations (1) or every iteration (0)
  long long nn;
  Coef<T> k;
  const void *mA;       // float32: the matrix-core product's A operand, or NULL for the
  float mscale;         //   vector-ALU product (then tx, ty, kz and nb_mv are its tiles')
  const T *E;
  const T *dinv;
  const uint8_t *mask;
  T *x, *r, *z, *q;
  T *p[CG_NP_MAX];
  double *cgp;          // [CGP_SIZE] block partials: p^T q, then r^T z and ||r||^2 by parity
  double *scal;         // [S_COUNT]
  int *flags;           // [F_COUNT]
};

// One block of a batched CG launch: its design (-1: padding, no work), its
// local block, and the design's partial-sum array, scalars, flags and the
// number of partials the kernel reads, so that one load gives a block
// everything its first loads need.
struct BlockEntry {
  double *cgp;
  double *scal;
  int *flags;
  int design, lb, nparts, pad_;
};

// Layout of CgDesc::cgp.  The product kernel of parity P reads the r^T z and
// ||r||^2 partials of set P^1 and writes the p^T q partials; the update
// kernel of parity P reads those and writes set P.
constexpr int CGP_PQ = 0;
constexpr int CGP_RZ = MAXB;          // + P * MAXB
constexpr int CGP_RR = 3 * MAXB;      // + P * MAXB
// bfloat16 z only (flexible CG with one-step orthogonalisation), written with
// r^T z (same parity): r_new^T p and z_new^T q partials.  Rounding z makes the
// Jacobi preconditioner vary from one iteration to the next, so the identities
// r_k^T p_(k-1) = 0 and beta = r^T z / (r^T z)_old no longer hold; the
// direction update beta = -z_new^T q_old / p_old^T q_old keeps consecutive
// directions K-conjugate, and the step length (r^T z + beta r^T p_old) /
// p^T K p is the exact line search along p.
constexpr int CGP_RP = 5 * MAXB;      // + P * MAXB
constexpr int CGP_ZQ = 7 * MAXB;      // + P * MAXB
constexpr int CGP_SIZE = 9 * MAXB;

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round-robin
// by block index.  xcd_local maps block b of nb to a local tile index such
// that every XCD gets one contiguous range of tiles: neighbouring tiles,
// which share halo node planes and elements, then share an L2.
constexpr int NXCD = 8;
__host__ __device__ inline int xcd_local(int b, int nb) {
  const int x = b % NXCD, slot = b / NXCD;
  const int base = nb / NXCD, extra = nb % NXCD;
  return x * base + (x < extra ? x : extra) + slot;
}

// Large product launches place their blocks in bands: XCD x (blocks b with
// b % 8 == x) takes a contiguous band of the x-y tiles of every z chunk,
// chunks in order, so all XCDs work in the same z slab at a time while
// neighbouring tiles still share an L2 (2-4% faster than one contiguous range
// of blocks per XCD at 256 x 128 x 128).  band_local returns the local block
// chunk * tiles + tile, or -1 for the padding blocks of the last, partial
// band; band_grid is the launch size.  Smaller launches keep xcd_local: there
// the padding costs more than the placement gains (6% per FP32 CG iteration
// at 96 x 48 x 48, and an FP64 grid beyond one round of resident blocks).
__host__ __device__ inline int band_local(int b, int tiles, int nchunks) {
  const int band = (tiles + NXCD - 1) / NXCD;
  const int x = b % NXCD, sl = b / NXCD;
  const int chunk = sl / band, tile = x * band + sl % band;
  return (tile < tiles && chunk < nchunks) ? chunk * tiles + tile : -1;
}
__host__ __device__ inline int band_grid(int tiles, int nchunks) {
  return NXCD * ((tiles + NXCD - 1) / NXCD) * nchunks;
}
constexpr int BAND_MIN_BLOCKS = 1536 / MV_BLOCK_SCALE;
// the product's local block of launch block b (or -1), and its launch size
__host__ __device__ inline int mv_local(int b, int tiles, int nchunks) {
  const int nb = tiles * nchunks;
  return nb >= BAND_MIN_BLOCKS ? band_local(b, tiles, nchunks) : xcd_local(b, nb);
}
__host__ __device__ inline int mv_grid(int tiles, int nchunks) {
  const int nb = tiles * nchunks;
  return nb >= BAND_MIN_BLOCKS ? band_grid(tiles, nchunks) : nb;
}

struct Grid {
  int nelx, nely, nelz;
  size_t nel, nn, ndof;
};

// ---------------------------------------------------------------- launchers
template <typename T, int MODE>
hipError_t launch_matvec(const MvArgs<T> &a, int *nblocks, hipStream_t s);
int matvec_kz(const Grid &g, bool fp64, bool mfma = false);
int matvec_blocks(const Grid &g, int kz, bool mfma = false);
// matrix-core float32 product (k_mfma.hip): the A operand for Poisson ratio
// nu (false when M = B + (lambda/mu) A is not exact in bfloat16), and the
// unit-cube scale mu / 72
bool mfma_operand_table(double nu, uint16_t out[2][64][8], float *mscale_unit);
hipError_t launch_matvec_mfma(const MvArgs<float> &a, int *nblocks, hipStream_t s);

hipError_t launch_modulus(const Grid &g, const double *x, double E0, double Emin, double penal,
                          double *E64, float *E32, int *flags, hipStream_t s);
hipError_t launch_diag(const Grid &g, const double *E64, double kd, const uint8_t *mask,
                       double *dinv64, float *dinv32, hipStream_t s);
hipError_t launch_mask_builtin(const Grid &g, int bc, uint8_t *mask, hipStream_t s);
hipError_t launch_load_builtin(const Grid &g, int bc, double load_total, const uint8_t *mask,
                               double *f, hipStream_t s);
hipError_t launch_mask_custom(const Grid &g, const uint8_t *dof_mask, uint8_t *mask, double *f,
                              hipStream_t s);

int vec_blocks(size_t nn);
// Start of an inner solve: r = b * scal[S_SCALE] (fixed DOFs 0), x = 0,
// z = D r, both directions 0, with the r^T z / ||r||^2 partials written
// (nb_up blocks, as the update kernel) to parity set `slot` of cgp.
template <typename T>
hipError_t launch_cg_init(const Grid &g, const double *b, const double *scal, T *x, T *r, T *z,
                          T *pA, T *pB, const T *dinv, const uint8_t *mask, double *cgp, int slot,
                          int nb_up, hipStream_t s, int zbf = 0,  // zbf: z stored in bfloat16
                          T *pC = nullptr, T *pD = nullptr);  // further direction slots (zeroed)
// One CG iteration for every design of a batch is the product kernel (with
// its last-block step length) followed by the update kernel (last-block beta
// and convergence test).  blockmaps: (design, local block) per block.
// One design, descriptor by value (the single-solve path).
template <typename T>
hipError_t launch_cg_matvec1(const CgDesc<T> &d, int slot, hipStream_t s,
                             hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
template <typename T>
hipError_t launch_cg_update1(const CgDesc<T> &d, int slot, hipStream_t s);
// `iters` CG iterations of one design as an instantiated graph (see k_matvec.hip)
template <typename T>
hipError_t build_cg_graph(const CgDesc<T> &d, int slot0, int iters, hipGraphExec_t *out);
template <typename T>
hipError_t build_cg_graph_batched(const CgDesc<T> *descs, const BlockEntry *bmv, int nb_mv,
                                  const BlockEntry *bup, int nb_up, int parity0, int iters,
                                  hipGraphExec_t *out);
template <typename T>
hipError_t launch_cg_matvec(const CgDesc<T> *descs, const BlockEntry *bmap_mv, int nb_mv, int parity,
                            hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr);
template <typename T>
hipError_t launch_cg_update(const CgDesc<T> *descs, const BlockEntry *bmap_up, int nb_up, int parity,
                            hipStream_t s);
int update_blocks(size_t nn);
// where the CG product gets z = D r: read as the update stored it, formed from
// r and the Jacobi diagonal, or as the descriptor's zfuse says (batched)
enum { ZF_READ = 0, ZF_FORM = 1, ZF_DESC = 2 };

// CG z = D r formed inside the product from this many nodes up (where the
// vectors stream from HBM); below, the update stores z and the product reads it
constexpr size_t ZFUSE_MIN_NODES = size_t(1) << 19;
int cg_zfuse(const Grid &g);

// u += (x + the pending grouped steps) / scal[S_SCALE]: the float64 solution
// update of the outer refinement.  With grouped x (xgroup) the steps since
// the last grouped update, sum_j alpha_j p[j] over j < (flags[F_SLOT0] +
// flags[F_ITERS] + 1) % np, are still pending and are applied here.
template <typename T>
hipError_t launch_axpy_out(const Grid &g, double *u, const T *d, const double *scal,
                           hipStream_t s, int np = 2, int xgroup = 0, T *const *p = nullptr,
                           const int *flags = nullptr);

hipError_t launch_finish_init(const double *cgp, int nb_up, int slot, double tol2_rel, int cap,
                              double *scal, int *flags, hipStream_t s, int slot0 = 0);
hipError_t launch_finish_sum(const double *part, int nb, int comp, double *scal, int idx,
                             hipStream_t s);
hipError_t launch_fill(void *p, size_t bytes, hipStream_t s);

// optimality-criteria update (k_oc.hip); scratch: OC_SCRATCH doubles
int oc_blocks(size_t nel);
// launches k0 .. k0 + count - 1 of the bisection (launch 0 starts the bracket)
hipError_t launch_oc_steps(const double *x, const double *dc, size_t nel, double move, double eta,
                           double target, double tol, double l2_0, int max_steps, double *scratch,
                           int k0, int count, int *flags, hipStream_t s);
// after k bisection launches: writes x_new and the output block
hipError_t launch_oc_apply(const double *x, const double *dc, double *xnew, size_t nel,
                           double move, double eta, double *scratch, int k, hipStream_t s);
hipError_t launch_set(double *p, size_t n, double v, hipStream_t s);

// shape derivative and Hilbertian extension (k_shape.hip).  The extension's
// CG keeps HCG_PQ_MAX + 4 x HCG_MAXB block partials, then 8 scalars.
constexpr int HCG_MAXB = 1024;
constexpr int HCG_PQ_MAX = 8192;
constexpr int HCG_SCAL_OFS = HCG_PQ_MAX + 4 * HCG_MAXB;
constexpr int HCG_SCRATCH = HCG_SCAL_OFS + 8;
// band: nel bytes of scratch (elements that meet |phi| <= eta)
hipError_t launch_shape_rhs(const Grid &g, const double *u, const double *phi, double h,
                            double lam, double mu, double eta, double c_s, double c_0,
                            uint8_t *band, double *contrib, double *out, hipStream_t s);
// iterations it0 .. it0 + count - 1 of the extension's CG (it0 == 0 also
// builds the Gamma_N mask from f and starts from x = 0); vec: r, z, p, q
hipError_t launch_hilbert(const Grid &g, double h, double ell, double rtol, int max_iters,
                          const double *f, const double *b, double *x, double *const vec[4],
                          uint8_t *gm, double *part, double *scal, int *flags, int it0, int count,
                          hipStream_t s);

// level-set evolution and reinitialisation (k_levelset.hip).  The largest
// |change| of a reinitialisation step is taken by atomic max over LS_SLOTS
// words on separate 128-byte lines (a block picks one by its index), so the
// atomics of thousands of blocks do not queue on one address; three such sets
// rotate between launches.  Scratch (8-byte words): the sets, then the loop
// state (3 doubles) and the max|v| word.
constexpr int LS_SLOTS = 64, LS_SLOT_STRIDE = 16;
constexpr int LS_SET_WORDS = LS_SLOTS * LS_SLOT_STRIDE;
constexpr int LS_STATE_OFS = 3 * LS_SET_WORDS;
constexpr int LS_VMAX_OFS = LS_STATE_OFS + 4;
constexpr int LS_SCRATCH = LS_STATE_OFS + 8;
hipError_t launch_ls_check(const Grid &g, const double *phi, const double *v, int *flags,
                           unsigned long long *vmax, hipStream_t s);
hipError_t launch_ls_advect(const Grid &g, double h, double dt, const double *in, const double *v,
                            double *out, hipStream_t s);
// launch k of the reinitialisation loop; slots: 3 sets, state: 3 doubles
hipError_t launch_ls_reinit(const Grid &g, double h, double dtau, double tol, int max_steps,
                            int k, const double *in, double *out, unsigned long long *slots,
                            double *state, hipStream_t s);
hipError_t launch_set_scale(double *scal, hipStream_t s);
hipError_t launch_dot(const double *a, const double *b, size_t n, double *part, int *nb,
                      hipStream_t s);

hipError_t launch_energy_sens(const Grid &g, const double *x, const double *u, const double *E64,
                              Coef<double> k, double E0, double Emin, double penal, double *dc,
                              double *part, int *nb, hipStream_t s);

hipError_t launch_filter(const Grid &g, int mode, int nofs, const int *ofs, const double *w,
                         double V, const double *x, const double *in, double *tmp, double *out,
                         hipStream_t s);

// SDF
hipError_t launch_node_mean(const Grid &g, const double *x, double *rho, hipStream_t s);
hipError_t launch_mt_count(const Grid &g, const double *rho, double rho_t, int *count,
                           hipStream_t s);
hipError_t launch_scan(const int *in, int *out, size_t n, int *block_sums, hipStream_t s);
hipError_t launch_mt_emit(const Grid &g, const double *rho, double rho_t, double h,
                          const int *offset, const int *count, double *tri, hipStream_t s);
// occ: scratch for the coarse occupancy bitmask, one bit per cell of
// ceil(nelx/4) ceil(nely/4) ceil(nelz/4) (at least ceil(cells / 32) ints)
hipError_t launch_udist(const Grid &g, double h, const int *count, const int *offset,
                        const double *tri, int *occ, const double *rho, double rho_t, double *phi,
                        hipStream_t s);
hipError_t launch_vf(const Grid &g, const double *phi, double *vf, hipStream_t s);
hipError_t launch_sign_inf(const Grid &g, const double *rho, double rho_t, double *phi,
                           hipStream_t s);

}  // namespace topo
