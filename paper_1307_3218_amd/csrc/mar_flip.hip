// Local flipping refinement of an eigenvector (Appendix).
//
// The components a_l of phi (level eps) change sign one at a time when that
// lowers R = |r|^2 (+ c p^2), r = (H - eps S) phi, p = phi_ref^T S phi. A flip
// of a_l changes r by -2 a_l (H - eps S) e_l on the rows of P(l) only (H and S
// are symmetric) and p by -2 a_l s_l, s = S phi_ref, so no product with the
// matrix is needed after the first residual. The rows are visited by colour of
// a distance-2 colouring of H's pattern, and in index order within a colour.
// Rows of one colour have disjoint column supports, so the |r|^2 part of each
// row's single-flip change does not depend on the colour's other flips: it is
// computed for all rows of the colour at once. Without the penalty the rows
// then decide at once. The penalty couples every row through p, so with it one
// wave walks the colour's rows in index order, each deciding on the p left by
// the flips before it: a sequential descent, every accepted flip lowering R.
// Sweeps repeat until one flips nothing or max_sweeps have run.
//
// One workgroup does everything (the refinement is a small cost next to the
// solve): the decisions and residual updates of a colour are spread over its
// threads, p and the flip count are kept in LDS, and every sum runs in a fixed
// order, with products and sums rounded separately (no fused multiply-add), so
// that every decision is reproducible.
#include "mar_device.h"
#include "mar_internal.h"

namespace mar {

constexpr int FLIP_WG = 1024;

__device__ __forceinline__ double bcast(double v, int t) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, t);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), t);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__global__ __launch_bounds__(FLIP_WG) void k_flip(int64_t M, const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ col, const double* __restrict__ hv,
                                                  const double* __restrict__ sv, double eps, double* phi,
                                                  const double* __restrict__ phi_ref, double cpen, int ncol,
                                                  const int32_t* __restrict__ coff, const int32_t* __restrict__ crow,
                                                  int max_sweeps, double* r, double* s, double* drr,
                                                  int8_t* flag,
                                                  double* __restrict__ Rout, int32_t* __restrict__ info) {
#pragma clang fp contract(off)
    const int tid = threadIdx.x;
    const bool pen = phi_ref != nullptr && cpen != 0.0;
    __shared__ double red[FLIP_WG];
    __shared__ double p_sh;
    __shared__ int nflip;
    // fixed-order sum of v over the workgroup (thread partials, then a tree)
    auto wg_sum = [&](double v) {
        red[tid] = v;
        __syncthreads();
        for (int w = FLIP_WG / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] = red[tid] + red[tid + w];
            __syncthreads();
        }
        const double t = red[0];
        __syncthreads();
        return t;
    };
    // first residual r = (H - eps S) phi and s = S phi_ref, each row in column order
    double rr = 0.0;
    for (int64_t i = tid; i < M; i += FLIP_WG) {
        double t = 0.0, u = 0.0;
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            const double a = hv[q] - eps * sv[q];
            t = t + a * phi[col[q]];
            if (pen) u = u + sv[q] * phi_ref[col[q]];
        }
        r[i] = t;
        if (pen) s[i] = u;
        rr = rr + t * t;
    }
    __threadfence_block();
    __syncthreads();
    if (tid == 0) {
        double p = 0.0;
        if (pen)
            for (int64_t l = 0; l < M; ++l) p = p + s[l] * phi[l];
        p_sh = p;
    }
    double R = wg_sum(rr);   // its barriers also publish p_sh
    if (tid == 0 && Rout) Rout[0] = R + (pen ? cpen * p_sh * p_sh : 0.0);
    int sweeps = 0;
    int64_t flips = 0;
    for (int sw = 0; sw < max_sweeps; ++sw) {
        if (tid == 0) nflip = 0;
        __syncthreads();
        for (int k = 0; k < ncol; ++k) {
            const int e0 = coff[k], e1 = coff[k + 1];
            // the |r|^2 part of each row's single-flip change, summed in the row's column order
            for (int e = e0 + tid; e < e1; e += FLIP_WG) {
                const int l = crow[e];
                const double a = phi[l];
                double d = 0.0;
                for (int q = rp[l]; q < rp[l + 1]; ++q) {
                    const double av = hv[q] - eps * sv[q];
                    d = d + av * ((4.0 * a) * a * av - (4.0 * a) * r[col[q]]);
                }
                if (pen)
                    drr[e] = d;
                else
                    flag[e] = d < 0.0 ? 1 : 0;
            }
            __threadfence_block();
            __syncthreads();
            if (pen && tid < 64) {
                // wave 0 walks the colour's rows in index order, 64 at a time: each
                // lane prepares its row's p-independent terms, then every lane takes
                // the same decisions on broadcast values, p carried in registers
                double p = p_sh;
                for (int base = e0; base < e1; base += 64) {
                    const int e = base + tid;
                    const bool in = e < e1;
                    double dl = 0.0, x = 0.0, y = 0.0, z = 0.0;
                    if (in) {
                        const int l = crow[e];
                        const double a = phi[l], sl = s[l];
                        dl = drr[e];
                        x = (4.0 * a) * a * sl * sl;
                        y = (4.0 * a) * sl;
                        z = (2.0 * a) * sl;
                    }
                    const int n = e1 - base < 64 ? e1 - base : 64;
                    int8_t mine = 0;
                    for (int t = 0; t < n; ++t) {
                        const double d = bcast(dl, t) + cpen * (bcast(x, t) - bcast(y, t) * p);
                        const bool f = d < 0.0;
                        if (f) p = p - bcast(z, t);
                        if (t == tid) mine = f ? 1 : 0;
                    }
                    if (in) flag[e] = mine;
                }
                if (tid == 0) p_sh = p;
            }
            __threadfence_block();
            __syncthreads();
            int mine = 0;
            for (int e = e0 + tid; e < e1; e += FLIP_WG) {
                if (!flag[e]) continue;
                const int l = crow[e];
                const double a = phi[l];
                for (int q = rp[l]; q < rp[l + 1]; ++q) {   // column l of a symmetric matrix: row l
                    const double av = hv[q] - eps * sv[q];
                    r[col[q]] = r[col[q]] - (2.0 * a) * av;
                }
                phi[l] = -a;
                ++mine;
            }
            if (mine) atomicAdd(&nflip, mine);
            __threadfence_block();
            __syncthreads();
        }
        double part = 0.0;
        for (int64_t i = tid; i < M; i += FLIP_WG) part = part + r[i] * r[i];
        R = wg_sum(part);
        const int nf = nflip;
        sweeps = sw + 1;
        flips += nf;
        if (tid == 0 && Rout) Rout[sw + 1] = R + (pen ? cpen * p_sh * p_sh : 0.0);
        __syncthreads();
        if (nf == 0) break;
    }
    if (tid == 0 && info) {
        info[0] = sweeps;
        info[1] = (int32_t)(flips < 0x7fffffff ? flips : 0x7fffffff);
    }
}

LaunchInfo launch_flip(int64_t M, const int32_t* rp, const int32_t* col, const double* hv, const double* sv,
                       double eps, double* phi, const double* phi_ref, double cpen, int ncol, const int32_t* coff,
                       const int32_t* crow, int max_sweeps, double* r, double* s, double* drr, int8_t* flag,
                       double* Rout, int32_t* info, hipStream_t st) {
    hipLaunchKernelGGL(k_flip, dim3(1), dim3(FLIP_WG), 0, st, M, rp, col, hv, sv, eps, phi, phi_ref, cpen, ncol,
                       coff, crow, max_sweeps, r, s, drr, flag, Rout, info);
    LaunchInfo li;
    li.wgs = 1;
    return li;
}

}  // namespace mar
