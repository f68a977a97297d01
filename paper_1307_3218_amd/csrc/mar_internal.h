// Internal declarations shared by the host API and the kernel launchers.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "mar.h"

namespace mar {

constexpr int WG = 256;            // threads per workgroup for every streaming kernel
constexpr int PROJ_Q = 8;          // 16-byte vectors per thread in a projection chunk
constexpr int PROJ_KG = 4;         // basis slabs reduced together in a projection
constexpr int MAX_ROW = 63;        // max stored entries in a row of H (|P(j)| <= 63)
constexpr int PROJR_Q = 4;         // 16-byte vectors per thread and right-hand side in a row tile
constexpr int PROJR_KG = 4;        // slabs owned by one workgroup in the delayed-schedule projection

// Row tiles per workgroup of the delayed-schedule projection: as many as keep
// the grid at about target_wgs workgroups (fewer partial sums), at least one.

// Grid of the delayed-schedule projection for nk slabs of nvec vectors: KG
// slabs per workgroup (nks splits), `tiles` row tiles per workgroup (as many
// as keep the grid near target_wgs), `groups` row groups. The partial-sum
// buffer needs groups * 3 * nk * B doubles. Used by the launcher and by the
// workspace sizing, so that both always agree.
struct ProjrGeom {
    int kg, q, nks;
    int64_t ntiles, tiles, groups;
};
// variant: 0 = 4 slabs x 4 vectors, 1 = 8 x 4, 2 = 4 x 4 non-temporal, 3 = 4 x 2, 4 = 8 x 2, 5 = 6 x 4,
// 6 = 6 x 2, 7 = 8 x 4 non-temporal (slabs per workgroup x 16-byte vectors per thread and row tile).
inline int projr_kg(int variant) {
    return variant == 1 || variant == 4 || variant == 7 ? 8 : (variant == 5 || variant == 6 ? 6 : 4);
}
inline int projr_q(int variant) { return variant == 3 || variant == 4 || variant == 6 ? 2 : PROJR_Q; }
// target_wgs (> 0) caps the grid: the row tiles are cut into target_wgs / nks
// groups, so that a grid of the device's resident capacity runs in one round
// and the partial sums stay few (groups * 3 * nk * B values).
inline ProjrGeom projr_geometry(int64_t nvec, int nk, int variant, int64_t target_wgs) {
    ProjrGeom g;
    g.kg = projr_kg(variant);
    g.q = projr_q(variant);
    g.nks = (nk + g.kg - 1) / g.kg;
    g.ntiles = (nvec + WG * g.q - 1) / (WG * g.q);
    int64_t groups = (target_wgs > 0 ? target_wgs : 1) / g.nks;
    groups = groups < 1 ? 1 : (groups > g.ntiles ? g.ntiles : groups);
    g.tiles = (g.ntiles + groups - 1) / groups;
    g.groups = (g.ntiles + g.tiles - 1) / g.tiles;
    return g;
}

// Device copy of one sparse matrix. BSR 4x4 (values [blk][r][c]) when the
// pattern has that structure, else CSR. Values are kept in FP64 and FP32.
struct DevMat {
    bool bsr = false;
    int64_t n = 0;          // block rows (BSR) or rows (CSR)
    int64_t nnz = 0;        // blocks (BSR) or entries (CSR)
    int32_t* ptr = nullptr; // n + 1
    int32_t* idx = nullptr; // nnz
    double* v64 = nullptr;  // nnz * (bsr ? 16 : 1)
    float* v32 = nullptr;
    int64_t span = 0;       // BSR: 90th percentile of |I - J| over the off-diagonal blocks (in a lattice, the
                            // distance to the neighbours in the next plane of cells; periodic wraps excluded)
    double bytes_per_pass(size_t p) const {  // values + indices read once
        return (double)nnz * ((bsr ? 16.0 : 1.0) * (double)p + 4.0) + (double)(n + 1) * 4.0;
    }
};

// Row tiles per chunk of the whole-cell block products' chunk-interleaved order (see xcd_chunk): 8 chunks
// span the matrix's typical far-neighbour distance; 0 (contiguous ranges per XCD) below 4 tiles.
inline int64_t spmm_chunk(int64_t span, int64_t tile_rows) {
    const int64_t c = span / (8 * tile_rows);
    return c >= 4 ? c : 0;
}

// Pointers of one seed block's device workspace.
template <typename T>
struct BlockWS {
    T* K;        // [nu][M][B]
    T* SK;       // [nu][M][B]
    T* W;        // [M][B]
    T* Z;        // [M][B]
    double* part;   // partial sums, [chunk][...]
    double* red1;   // [2][nu][B]  (h column, c1)
    double* red2;   // [nu][B]     (c2)
    double* redb;   // [B]         (beta^2)
    double* h;      // [B][nu][nu]
    double* beta;   // [B]
    int32_t* active;   // [B]
    int32_t* nu_eff;   // [B]
};

// ---- launchers (defined per element type in mar_launch_*.hip) ----
// Every launcher returns the number of workgroups it launched (for partials)
// and sets *bytes / *flops to the algorithmic traffic of the launch.
struct LaunchInfo {
    int64_t wgs = 0;    // -1: not launched, the partial-sum buffer is too small
    double bytes = 0, flops = 0;
};

template <typename T>
LaunchInfo launch_init(int B, int64_t Mp, int64_t M, const int32_t* seeds, int nseeds, const double* diagS,
                       int nu, T* K0, int32_t* active, int32_t* nu_eff, double* uu, hipStream_t s);
// ndot = 0: Y = A X; 1: also partial sums of X.Y per seed; 2: X.Y and X.X (part[wg][d][b]).
// part_cap: doubles available at part (checked before launch).
// tdist (optional, BSR and B >= vector width only): tile distances; tiles with tdist > lim are skipped (their
// outputs are not written, their partials are zero).
// mask (optional, BSR and B >= vector width only): local-region bits per block row (W words); the product
// is kept only on the rows inside each seed's region.
// rdist (optional, BSR and B >= vector width only): block-row distances; rows with rdist > lim are written as
// zero without reading X (the same for launch_spmm2).
template <typename T>
LaunchInfo launch_spmm(int B, const DevMat& A, const T* X, T* Y, double* part, int ndot, int64_t part_cap,
                       hipStream_t s, const int32_t* tdist = nullptr, int lim = 0, const uint32_t* mask = nullptr,
                       int W = 0, const int32_t* rdist = nullptr);
template <typename T>
// stride: elements between consecutive basis slabs (>= M * B).
LaunchInfo launch_proj(int B, int ns, const T* b0, const T* b1, int64_t M, int64_t stride, int nk, const T* x,
                       double* part, int64_t part_cap, int64_t* nchunks, hipStream_t s);
template <typename T>
LaunchInfo launch_upd(int B, const T* basis, int64_t M, int64_t stride, int nk, const double* c, T* x,
                      hipStream_t s);
template <typename T>
LaunchInfo launch_append(int B, int64_t M, const T* W, const T* Z, const double* beta,
                         const int32_t* active, T* Kn, T* SKn, hipStream_t s);
// Rows K[P(j), :] of the block's seeds into Kp[(b * nu + k) * max_row + t] (FP64) and nu_eff into nu_copy.
template <typename T>
LaunchInfo launch_gather(int B, int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff_blk, const T* K,
                         int64_t stride, const int32_t* Hrp, const int32_t* Hcol, int max_row, double* Kp,
                         int32_t* nu_copy, hipStream_t s);
// Eigen-state modes of the subspace eigensolver (Sec. 3, Eq. 3; Appendix).
struct EigExtra {
    int mode = 0;                 // 0: assembly (or kept rows); 1: full eigenvectors; 2: signed Eq. 3 component
    double* Rg = nullptr;         // mode 1: R in global memory, [seed][nu][nu + 1]
    double* Y = nullptr;          // mode 1: y_alpha of each seed, [seed][alpha][nu]
    const double* pref = nullptr; // mode 2: K^T v_ref, [k][pB]
    int pB = 1;
    const double* win = nullptr;  // mode 2: {eps_k, eta(k-1), eta(k)} on the device
    double sigma = 0.0;           // mode 2: width of the smoothed delta
    double* phi = nullptr;        // mode 2: e_j^T phi_k of each seed
    int eig_max_sweeps = 40;      // Jacobi sweeps allowed
};
// nu_eff of a seed whose subspace eigensolve did not converge
constexpr int NU_NOCONV = -3;
LaunchInfo launch_eig(int nseeds, const int32_t* seeds, int nu, double* h, const int32_t* nu_eff_blk,
                      const double* Kp, const int32_t* Hrp, const int32_t* Hcol, const double* Hval,
                      const double* SvalH, const double* diagS, int max_row, double mu, double kT, double* rho,
                      double* e_seed, double* n_seed, int32_t* nu_eff_out, double* eps_out, double* w_out,
                      double* zc, const EigExtra& ex, hipStream_t s);
// zc != nullptr: k_eig keeps zc[(b*nu + alpha)*max_row + t] = e_i.v_alpha (i = P(j)[t]) and writes levels
// and weights (eps_out, w_out required) instead of assembling; k_assemble finishes at mu = *mu.
constexpr int MAX_NU_ASSEMBLE = 4096;
LaunchInfo launch_assemble(int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff, const double* eps,
                           const double* zc, int max_row, const int32_t* Hrp, const int32_t* Hcol,
                           const double* Hval, const double* SvalH, const double* mu, double kT, double* rho,
                           double* e_seed, double* n_seed, hipStream_t s);
// Eigen states: bisection of the smoothed integrated density of states for the counts k - 1, k - 1/2, k
// (lv = {eta(k - 1/2), eta(k - 1), eta(k)}); part >= 3 * 512 doubles, st >= 6 doubles.
LaunchInfo launch_dos_search(int64_t nseeds, int nu, const int32_t* nu_eff, const double* eps, const double* w,
                             double sigma, int k, int iters, double* part, double* st, double* lv, hipStream_t s);
// The seed and subspace eigenvector with the largest |(e_j.v_alpha) window| (ref = {position, alpha, seed}).
LaunchInfo launch_es_reference(int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff, const double* eps,
                               const double* zc, int max_row, const int32_t* Hrp, const int32_t* Hcol,
                               const double* lv, double sigma, double* cmax, int32_t* amax, int32_t* ref,
                               int32_t* refseed, hipStream_t s);
// Reference seed solved alone (B = 1): y_ref among its eigenvectors Y, then v_ref = K y_ref (M doubles).
template <typename T>
LaunchInfo launch_es_refvec(const T* K, int64_t stride, int64_t M, const int32_t* seed, int nu,
                            const int32_t* nu_eff, const double* Y, const double* eps, const double* lv, double sigma,
                            double* yref, double* vref, hipStream_t s);
// part[(g * nu + k) * B + b] = sum over row chunk g of K[k][i][b] vref[i]; chunks of rows, G groups.
template <typename T>
LaunchInfo launch_es_pdot(int B, const T* K, int64_t stride, int64_t M, int64_t Mp, int nu, const double* vref,
                          double* part, int groups, hipStream_t s);
// Bisection for the Fermi level over the levels of nseeds seeds; part >= 2 * 512 doubles, st = {lo, hi, mu};
// the final mu is also written to *mu_out when mu_out != nullptr.
LaunchInfo launch_fermi_search(int64_t nseeds, int nu, const int32_t* nu_eff, const double* eps, const double* w,
                               double n_target, double kT, int iters, double* part, double* st, double* mu_out,
                               hipStream_t s);

// Y = H X and Z = S X in one pass (SH: S's values on H's BSR pattern); refused (wgs = -1) unless H is BSR
// and B >= the vector width. ndot as in launch_spmm, against Z.
template <typename T>
LaunchInfo launch_spmm2(int B, const DevMat& H, const DevMat& SH, const T* X, T* Y, T* Z, double* part, int ndot,
                        int64_t part_cap, hipStream_t s, const int32_t* tdist = nullptr, int lim = 0,
                        const uint32_t* mask = nullptr, int W = 0, const int32_t* rdist = nullptr);
// Local regions: the dual product, S y and the update over the row tiles of the support list (entries
// [0, cnt[lim])) in a grid-stride loop of `grid` workgroups; spmm2 partials are per workgroup (grid slots).
template <typename T>
LaunchInfo launch_spmm2_list(int B, const DevMat& H, const DevMat& SH, const T* X, T* Y, T* Z, double* part,
                             int ndot, int64_t part_cap, const int32_t* list, const int32_t* cnt, int lim,
                             const uint32_t* mask, int W, int64_t grid, hipStream_t s);
template <typename T>
LaunchInfo launch_spmm_list(int B, const DevMat& A, const T* X, T* Y, const int32_t* list, const int32_t* cnt,
                            int lim, const uint32_t* mask, int W, int64_t grid, hipStream_t s);
// The dual update over the support list in distance order (entries [0, cnt[lim]), grid workgroups in a
// grid-stride loop; nt: non-temporal slab loads). With want_w, the entries [cnt[lim], cnt[limz]) (limz > lim)
// get zeros in wout.
template <typename T>
LaunchInfo launch_upd2_list(int B, T* basis, int64_t M, int64_t stride, int n, const T* cA, const T* cB,
                            const double* gam, const double* Fn, const T* y, T* wout, bool want_w,
                            const int32_t* list, const int32_t* Dl, const int32_t* cnt, int lim, int limz,
                            int64_t grid, bool nt, hipStream_t s, bool acc64 = false);
// Zero the row tiles within hmax + 1 hops of a block's seeds (one more BFS level on dist, which holds the levels
// up to hmax) in nsl slabs of slab_bytes from base and in y; tiles are 4 * WG vectors of 16 bytes, nvec per slab.
LaunchInfo launch_zero_ring(int64_t nbrow, const int32_t* brp, const int32_t* bcol, int32_t* dist, int hmax,
                            int bpt, void* base, int64_t slab_bytes, int nsl, void* y, int64_t nvec, hipStream_t s);
// Delayed-reorthogonalization schedule.
// Projection sweep (variants as in projr_geometry); target_wgs > 0.
template <typename T>
LaunchInfo launch_projr(int B, const T* basis, int64_t M, int64_t stride, int nk, const T* r0, const T* r1,
                        const T* r2, double* part, int64_t part_cap, int64_t* ngroups, int64_t target_wgs,
                        int variant, hipStream_t s);
// Workgroups of that projection kernel one compute unit holds at once (>= 1).
template <typename T>
int projr_blocks_per_cu(int B, int variant);
// Slab bytes per update sweep above which the slab loads are non-temporal: twice the 256 MB last-level
// (Infinity) cache, so that a basis that fits in it keeps being served from it.
constexpr double kNtSweepBytes = 512.0 * 1024 * 1024;
// cA/cB: [n][B] coefficients in the basis precision T.
// upd_q: 16-byte vectors per thread (2, 4 or 8; 0 = 4), reduced for small grids. Every row of every slab
// (with support tracking the update runs over the tile list instead: launch_upd2_list).
// acc64 (FP32 basis): the running sums over the slabs in FP64, rounded once when stored.
template <typename T>
LaunchInfo launch_upd2(int B, T* basis, int64_t M, int64_t stride, int n, const T* cA, const T* cB,
                       const double* gam, const double* Fn, const T* y, T* wout, bool want_w, int upd_q,
                       hipStream_t s, bool acc64 = false);
// Subspace dimension above which the FP32 form's update keeps its running sums in FP64. At nu = 300 on the
// 1048576-row lattice they halve the form's rho error against the oracle; switched on at nu = 100 on the
// 131072-row lattice, where FP32 sums already meet the form's bar with room, they cost 0.7 % of the rate.
constexpr int kUpdAcc64Nu = 128;
// cAf/cBf (optional): the update coefficients rounded to FP32 for an FP32 basis.
// redb (n >= 1): {u~.S u~ [B], u~.u~ [B]} of slab n; the kernel first takes the breakdown test of slab n and
// sets BT, UU.
LaunchInfo launch_coef(int B, int nu, int n, const double* red, double* A, double* G, double* R, double* C1,
                       double* BT, double* UU, double* cA, double* cB, float* cAf, float* cBf,
                       double* gam, double* Fn, int32_t* active, int32_t* nu_eff, double tau, const double* redb,
                       hipStream_t s);

// Fixed-order sums out[o] = sum_c part[c * L + o]. With tmp (tmp_cap doubles, not read by anything in flight)
// and many chunks onto few outputs, the sum runs in two stages through tmp.
LaunchInfo launch_reduce(const double* part, int64_t nchunks, int64_t L, double* out, double* h, int B, int nu,
                         int n, hipStream_t s, double* tmp = nullptr, int64_t tmp_cap = 0);

// ---- support tracking of a seed block (exact zeros of the Krylov vectors) ----
constexpr int32_t SUP_FAR = 0x3fffffff;   // tile distance: farther than the largest hop count kept
// BFS over H's block pattern from the block rows of the seeds (hmax levels), tile distances D (bpt block rows
// per tile, ceil(nbrow / bpt) tiles), cnt[h] = tiles with D <= h (h = 0..hmax), and the tiles with D <= hmax
// sorted by (D, index) into list (Dl: their D).
// Distances above hmax count as SUP_FAR (never nonzero); cnt has hcnt + 1 entries (hcnt >= hmax).
LaunchInfo launch_support(int64_t M, int64_t nbrow, const int32_t* brp, const int32_t* bcol, int64_t nnzb,
                          const int32_t* seeds, int ns, int bpt, int hmax, int hcnt, int32_t* dist, int32_t* D,
                          int32_t* cnt, int32_t* list, int32_t* Dl, hipStream_t s);
// Local regions: per block row, W = ceil(B / 32) words whose bit b says the row is within r hops of seed b's
// block; m0, m1 hold nbrow * W words each; returns the buffer that holds the result.
const uint32_t* launch_local_masks(int64_t M, int64_t nbrow, const int32_t* brp, const int32_t* bcol,
                                   const int32_t* seeds, int ns, int W, int r, uint32_t* m0, uint32_t* m1,
                                   hipStream_t s);
// Work plan of the support-restricted projection of step n: 8 + 4 * grid ints, grid = G + chunks.
__host__ __device__ inline int64_t projr_sp_grid(int64_t G, int nk, int kg) { return G + (nk + kg - 1) / kg; }
// The plans of steps n0 .. n0 + nsteps - 1 in one launch, step n0 + i at plans + i * pstride (pstride >= the
// largest plan; refused otherwise).
LaunchInfo launch_projr_plan(const int32_t* cnt, const int32_t* Dl, int n0, int nsteps, int kg, int64_t G,
                             int64_t pstride, int32_t* plans, hipStream_t s);
// Fixed-order sum of the per-workgroup partials of that projection into red[3][nk][B].
LaunchInfo launch_reduce_sp(const double* part, const int32_t* plan, int64_t grid, int kg, int nk, int B,
                            double* out, hipStream_t s);
// The projection sweep over the planned tiles (variants as in projr_geometry); partials part[wg][3][kg][B].
template <typename T>
LaunchInfo launch_projr_sp(int B, const T* basis, int64_t M, int64_t stride, int n, const T* r0, const T* r1,
                           const T* r2, const int32_t* list, const int32_t* cnt, const int32_t* plan, int64_t grid,
                           double* part, int64_t part_cap, int variant, hipStream_t s);
LaunchInfo launch_norm(int B, int nk, const double* beta2, const double* c1, const double* c2, double tau,
                       int32_t* active, int32_t* nu_eff, double* beta, int n, hipStream_t s);
LaunchInfo launch_sum(const double* x, int64_t n, double* out, hipStream_t s);
LaunchInfo launch_zero(void* p, int64_t bytes, hipStream_t s);  // bytes: multiple of 16

// Local flipping refinement (Appendix), one workgroup: phi [M] in/out; colours: ncol lists, rows crow[coff[k]..
// coff[k+1]) in index order; r, s [M] and flag [M] workspace; Rout [max_sweeps + 1] and info [2] optional.
LaunchInfo launch_flip(int64_t M, const int32_t* rp, const int32_t* col, const double* hv, const double* sv,
                       double eps, double* phi, const double* phi_ref, double cpen, int ncol, const int32_t* coff,
                       const int32_t* crow, int max_sweeps, double* r, double* s, double* drr, int8_t* flag,
                       double* Rout, int32_t* info, hipStream_t st);

// Largest B accepted for an element type (P = B / vector width must fit one wavefront).
template <typename T>
constexpr int max_block() { return sizeof(T) == 4 ? 256 : 128; }

size_t eig_lds_bytes(int nu, int max_row, bool a_in_lds);
bool eig_a_fits_lds(int nu, int max_row);

// The device a context lives on (-1 for NULL).
int ctx_device(const mar_ctx* c);
// Record msg as the context's last error and return st.
mar_status ctx_error(mar_ctx* c, mar_status st, const char* msg);
// mar_solve_async on the caller's workspace ws[0, ws_bytes): no device allocation. The batched form's
// planned seed block (when the tuning fixes none) is halved until the workspace fits; MAR_ERR_ARG when
// even the smallest block does not fit.
mar_status solve_async_ext(mar_ctx* c, const int32_t* d_seeds, int64_t n_seeds, int32_t nu, double mu, double kT,
                           mar_precision prec, mar_form form, double* d_rho, double* d_e_band, double* d_e_seed,
                           double* d_n_seed, int32_t* d_nu_eff, double* d_eps, double* d_weight, void* ws,
                           size_t ws_bytes, void* hip_stream);

}  // namespace mar
