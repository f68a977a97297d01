// Type-independent FP64 kernels: fixed-order reduction of partial sums, the
// norm / breakdown decision of one Gram-Schmidt step, and the energy sum.
#include <algorithm>

#include "mar_device.h"
#include "mar_internal.h"

namespace mar {

// out[o] = sum_c part[c * L + o] for o < L, summed in a fixed order (chunk
// lanes strided by CL, then the CL lane sums in order). When h != nullptr the
// first nk*B outputs are also the subspace-matrix column n: o = k * B + b is
// written to h[b][k][n].
template <int OPW>
__global__ __launch_bounds__(WG) void k_reduce(const double* __restrict__ part, int64_t nchunks, int64_t L,
                                               double* __restrict__ out, double* __restrict__ h, int B, int nu,
                                               int n, int64_t hL) {
    constexpr int CL = WG / OPW;  // chunk lanes
    const int oi = threadIdx.x % OPW, cl = threadIdx.x / OPW;
    const int64_t o = (int64_t)blockIdx.x * OPW + oi;
    double s0 = 0.0, s1 = 0.0;
    if (o < L) {
        int64_t c = cl;
        for (; c + CL < nchunks; c += 2 * CL) {
            s0 += part[c * L + o];
            s1 += part[(c + CL) * L + o];
        }
        if (c < nchunks) s0 += part[c * L + o];
    }
    __shared__ double lds[WG];
    lds[threadIdx.x] = s0 + s1;
    __syncthreads();
    if (cl == 0 && o < L) {
        double t = 0.0;
        for (int k = 0; k < CL; ++k) t += lds[k * OPW + oi];
        out[o] = t;
        if (h != nullptr && o < hL) {
            const int64_t k = o / B, b = o % B;
            h[(b * nu + k) * (int64_t)nu + n] = t;
        }
    }
}

// First stage of a two-stage reduction of many chunks onto few outputs:
// tmp[y * L + o] = sum of part[c * L + o] over the chunks c of range y
// (chunks [y * cps, (y + 1) * cps)), four chunk lanes of 64 outputs per
// workgroup, each lane's chunks in order with four running sums, then the
// lanes in order. Rows of 64 consecutive outputs are read whole.
__global__ __launch_bounds__(WG) void k_reduce_split(const double* __restrict__ part, int64_t nchunks, int64_t L,
                                                     int64_t cps, double* __restrict__ tmp) {
    const int oi = threadIdx.x % 64, cl = threadIdx.x / 64;
    const int64_t o = (int64_t)blockIdx.x * 64 + oi;
    const int64_t c0 = (int64_t)blockIdx.y * cps;
    const int64_t c1 = c0 + cps < nchunks ? c0 + cps : nchunks;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (o < L) {
        int64_t c = c0 + cl;
        for (; c + 12 < c1; c += 16) {
            s0 += part[c * L + o];
            s1 += part[(c + 4) * L + o];
            s2 += part[(c + 8) * L + o];
            s3 += part[(c + 12) * L + o];
        }
        for (; c < c1; c += 4) s0 += part[c * L + o];
    }
    __shared__ double lds[WG];
    lds[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (cl == 0 && o < L)
        tmp[(int64_t)blockIdx.y * L + o] = ((lds[oi] + lds[64 + oi]) + lds[128 + oi]) + lds[192 + oi];
}

LaunchInfo launch_reduce(const double* part, int64_t nchunks, int64_t L, double* out, double* h, int B, int nu,
                         int n, hipStream_t s, double* tmp, int64_t tmp_cap) {
    const int64_t hL = h ? (int64_t)(n + 1) * B : 0;
    LaunchInfo li;
    // Many chunks onto few outputs (the per-workgroup partials of a product kernel): split the chunks into
    // ranges of RED_CPS, reduce each range over whole rows, then the range sums in order.
    constexpr int64_t RED_CPS = 128;
    const int64_t nsplit = (nchunks + RED_CPS - 1) / RED_CPS;
    if (tmp != nullptr && nchunks >= 8 * RED_CPS && L <= 4096 && nsplit * L <= tmp_cap) {
        const dim3 grid((unsigned)((L + 63) / 64), (unsigned)nsplit);
        hipLaunchKernelGGL(k_reduce_split, grid, dim3(WG), 0, s, part, nchunks, L, RED_CPS, tmp);
        const int64_t wgs = (L + 3) / 4;
        hipLaunchKernelGGL((k_reduce<4>), dim3(wgs), dim3(WG), 0, s, tmp, nsplit, L, out, h, B, nu, n, hL);
        li.wgs = (int64_t)grid.x * grid.y + wgs;
        li.bytes = (double)(nchunks + 2 * nsplit + 1) * L * 8.0;
        li.flops = (double)nchunks * L;
        return li;
    }
    if (L <= 2048) {
        const int64_t wgs = (L + 3) / 4;
        hipLaunchKernelGGL((k_reduce<4>), dim3(wgs), dim3(WG), 0, s, part, nchunks, L, out, h, B, nu, n, hL);
        li.wgs = wgs;
    } else {
        const int64_t wgs = (L + 15) / 16;
        hipLaunchKernelGGL((k_reduce<16>), dim3(wgs), dim3(WG), 0, s, part, nchunks, L, out, h, B, nu, n, hL);
        li.wgs = wgs;
    }
    li.bytes = (double)(nchunks + 1) * L * 8.0;
    li.flops = (double)nchunks * L;
    return li;
}

// Norm and breakdown of the new residual of each seed (all in FP64):
//   beta = sqrt(w^T S w), eta^2 = |c1|^2 + |c2|^2 + beta^2,
//   breakdown if beta <= tau * eta -> nu_eff = n + 1 and the seed stops;
//   w^T S w < 0 (or not finite) -> nu_eff = -1 (S not positive definite).
__global__ __launch_bounds__(WG) void k_norm(int B, int nk, const double* __restrict__ beta2,
                                             const double* __restrict__ c1, const double* __restrict__ c2,
                                             double tau, int32_t* __restrict__ active, int32_t* __restrict__ nu_eff,
                                             double* __restrict__ beta, int n) {
    // thread (part, b): partial sums of |c1|^2 + |c2|^2 over k = part, part + np, ...
    __shared__ double lds[WG];
    const int np = WG / B;
    const int b = threadIdx.x % B, part = threadIdx.x / B;
    double s = 0.0;
    if (part < np)
        for (int k = part; k < nk; k += np) {
            const double a1 = c1[(int64_t)k * B + b], a2 = c2[(int64_t)k * B + b];
            s += a1 * a1 + a2 * a2;
        }
    lds[threadIdx.x] = s;
    __syncthreads();
    if ((int)threadIdx.x >= B) return;
    double cc = 0.0;
    for (int q = 0; q < np; ++q) cc += lds[q * B + b];
    if (!active[b]) {
        beta[b] = 0.0;
        return;
    }
    const double bb = beta2[b];
    if (!(bb >= 0.0) || !(bb < INFINITY)) {
        nu_eff[b] = -1;
        active[b] = 0;
        beta[b] = 0.0;
        return;
    }
    const double bt = sqrt(bb);
    const double eta = sqrt(cc + bb);
    if (bt <= tau * eta) {
        nu_eff[b] = n + 1;
        active[b] = 0;
        beta[b] = 0.0;
    } else {
        beta[b] = bt;
    }
}

LaunchInfo launch_norm(int B, int nk, const double* beta2, const double* c1, const double* c2, double tau,
                       int32_t* active, int32_t* nu_eff, double* beta, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_norm, dim3(1), dim3(WG), 0, s, B, nk, beta2, c1, c2, tau, active, nu_eff, beta, n);
    LaunchInfo li;
    li.wgs = 1;
    li.bytes = (2.0 * nk + 3.0) * B * 8.0;
    return li;
}

// out = sum of x[0..n) in a fixed order (strided lane sums, then a tree).
__global__ __launch_bounds__(WG) void k_sum(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
    __shared__ double lds[WG];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += WG) s += x[i];
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int w = WG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = lds[0];
}

LaunchInfo launch_sum(const double* x, int64_t n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(WG), 0, s, x, n, out);
    LaunchInfo li;
    li.wgs = 1;
    li.bytes = (double)(n + 1) * 8.0;
    return li;
}

// Zero n16 16-byte words (the padded rows of the work vectors, and the basis
// of a seed block under support tracking; a kernel rather than a memset so the
// sequence stays capturable). A grid-stride loop over a bounded grid: a launch
// must stay below 2^32 work-items, and the basis of the largest instance is
// 80 GB (5e9 words).
constexpr int64_t ZERO_MAX_WGS = 16384;
__global__ __launch_bounds__(WG) void k_zero(double2* __restrict__ p, int64_t n16) {
    const int64_t step = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n16; i += step) p[i] = make_double2(0.0, 0.0);
}

LaunchInfo launch_zero(void* p, int64_t bytes, hipStream_t s) {
    const int64_t n16 = bytes / 16;
    const int64_t need = (n16 + WG - 1) / WG;
    const int64_t wgs = need < ZERO_MAX_WGS ? need : ZERO_MAX_WGS;
    LaunchInfo li;
    if (wgs > 0) hipLaunchKernelGGL(k_zero, dim3((unsigned)wgs), dim3(WG), 0, s, (double2*)p, n16);
    li.wgs = wgs;
    li.bytes = (double)bytes;
    return li;
}

// ---------------------------------------------------------------------------
// Delayed-reorthogonalization schedule: small FP64 per-seed algebra of step n.
//
// Entering step n, u_0..u_{n-1} are final (K^T S K = I) and u~ (slab n) has
// had one Gram-Schmidt pass and unit S-norm; y = H u~. The projection sweep
// gave, per seed, c2 = K^T S u~ (second-pass coefficients of u~), g = K^T S y,
// e = K^T y, and the self products u~.S y, u~.y. With
//   gamma = sqrt(1 - |c2|^2),  u_n = (u~ - K c2) / gamma,
// and the relation H K = K R collected from earlier steps (R upper Hessenberg
// of the Gram-Schmidt coefficients, column n-1 completed here), this kernel
// produces
//   column n of A = K^T H K:  A[:n+1, n] = (E - G q) / gamma,  q = R c2,
//     E = [e ; (u~.y - c2.e) / gamma],  G the Euclidean Gram matrix K^T K;
//   column n of G from t = K^T u~ = (A[:n, n-1] - G c1_prev) / beta~_prev;
//   the first-pass coefficients of H u_n against the S-basis,
//     c1 = (F - q) / gamma,  F = [g ; (u~.S y - c2.g) / gamma];
//   and the update coefficients (c2, g, gamma, F_n) for k_upd2.
// The final norm of the vector appended at step n-1 is beta~_prev * gamma; it
// is tested here against tau * eta (eta^2 = |c1_prev|^2 + beta~_prev^2 (|c2|^2 +
// gamma^2)), the same test the two-pass schedule applies, one step later.
// Slab n holds u~ unnormalized, s u~ with s = beta~_prev (1 at n = 0), and so
// do the sweep's right-hand sides; the products are rescaled here, and the
// update coefficients go out multiplied by s (k_upd2 divides by s gamma).
// A stopped seed gets gamma = inf, so that its slabs become zero.
// One workgroup per seed; A is h[b][k][n]; G is [nu][nu]; R is column-major
// [nu][nu+1] (R_{p,k} at k*(nu+1) + p).
__global__ __launch_bounds__(WG) void k_coef(int B, int nu, int n, const double* __restrict__ red,
                                             double* __restrict__ Ah, double* __restrict__ Gm,
                                             double* __restrict__ Rm, double* __restrict__ C1,
                                             double* __restrict__ BT, double* __restrict__ UU,
                                             double* __restrict__ cA, double* __restrict__ cB,
                                             float* __restrict__ cAf, float* __restrict__ cBf,
                                             double* __restrict__ gam, double* __restrict__ Fn,
                                             int32_t* __restrict__ active, int32_t* __restrict__ nu_eff, double tau,
                                             const double* __restrict__ redb) {
    extern __shared__ double sm[];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int nk = n + 1;
    double* c2 = sm;
    double* g = c2 + (nu + 1);
    double* e = g + (nu + 1);
    double* c1p = e + (nu + 1);
    double* t = c1p + (nu + 1);
    double* gc2 = t + (nu + 1);
    double* q = gc2 + (nu + 1);
    double* gq = q + (nu + 1);
    double* red8 = gq + (nu + 1);
    double* hsum = red8 + 8;   // [WG][3]: the two halves' sums of the Gram pass
    auto bsum = [&](double v) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        __syncthreads();
        if ((tid & 63) == 0) red8[tid >> 6] = v;
        __syncthreads();
        return (red8[0] + red8[1]) + (red8[2] + red8[3]);
    };
    auto stop = [&](int nu_new) {
        for (int k = tid; k < n; k += WG) {
            cA[(int64_t)k * B + b] = 0.0;
            cB[(int64_t)k * B + b] = 0.0;
            if (cAf) {
                cAf[(int64_t)k * B + b] = 0.0f;
                cBf[(int64_t)k * B + b] = 0.0f;
            }
        }
        if (tid == 0) {
            gam[b] = INFINITY;
            Fn[b] = 0.0;
            if (nu_new >= 0) {
                nu_eff[b] = nu_new;
                active[b] = 0;
            }
        }
    };
    // Step n >= 1 (redb != nullptr): first the breakdown test of slab n, the unnormalized residual of step
    // n - 1, from redb = {u~.S u~ [B], u~.u~ [B]}: beta~ = sqrt(u~.S u~) <= tau sqrt(|c1_prev|^2 + beta~^2)
    // stops the seed at nu_eff = n; a negative or non-finite u~.S u~ flags S as not positive definite
    // (nu_eff = -1). Otherwise beta~ and u~.u~ / beta~^2 become BT and UU.
    double btp = BT[b], uu = UU[b];
    if (redb != nullptr) {
        double s2 = 0.0;
        for (int k = tid; k < n; k += WG) {
            const double a = C1[(int64_t)b * nu + k];
            s2 += a * a;
        }
        const double bb = redb[b], ww = redb[B + b], cc = bsum(s2);
        if (active[b]) {
            int nu_new = 0;
            const bool bad = !(bb >= 0.0) || !(bb < INFINITY);
            if (bad) nu_new = -1;
            else if (sqrt(bb) <= tau * sqrt(cc + bb)) nu_new = n;
            if (bad || nu_new == n) {
                if (tid == 0) {
                    nu_eff[b] = nu_new;
                    active[b] = 0;
                    BT[b] = 0.0;
                }
                stop(-1);
                return;
            }
            btp = sqrt(bb);
            uu = ww / bb;
            if (tid == 0) {
                BT[b] = btp;
                UU[b] = uu;
            }
        }
    }
    if (!active[b]) {
        stop(-1);
        return;
    }
    double* A = Ah + (int64_t)b * nu * nu;
    double* G = Gm + (int64_t)b * nu * nu;
    double* Rc = Rm + (int64_t)b * nu * (nu + 1);
    const double sc = n >= 1 ? btp : 1.0;   // scale of slab n
    for (int k = tid; k < n; k += WG) {
        c2[k] = red[((int64_t)0 * nk + k) * B + b] / sc;
        g[k] = red[((int64_t)1 * nk + k) * B + b] / sc;
        e[k] = red[((int64_t)2 * nk + k) * B + b] / sc;
        c1p[k] = C1[(int64_t)b * nu + k];
    }
    const double utsy = red[((int64_t)1 * nk + n) * B + b] / sc / sc;
    const double uty = red[((int64_t)2 * nk + n) * B + b] / sc / sc;
    __syncthreads();
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
    for (int k = tid; k < n; k += WG) {
        p0 += c2[k] * c2[k];
        p1 += c1p[k] * c1p[k];
        p2 += c2[k] * e[k];
        p3 += c2[k] * g[k];
    }
    const double s_cc = bsum(p0), s_c1p = bsum(p1), s_ce = bsum(p2), s_cg = bsum(p3);
    const double gam2 = 1.0 - s_cc;
    if (!(gam2 > 0.0)) {  // u~ lies in span(K): the Krylov space is exhausted
        stop(n);
        return;
    }
    const double gm = sqrt(gam2);
    if (n >= 1) {
        const double bf = btp * gm;
        const double eta = sqrt(s_c1p + btp * btp * (s_cc + gam2));
        if (bf <= tau * eta) {
            stop(n);
            return;
        }
        for (int p = tid; p < n; p += WG) Rc[(int64_t)(n - 1) * (nu + 1) + p] = c1p[p] + btp * c2[p];
        if (tid == 0) Rc[(int64_t)(n - 1) * (nu + 1) + n] = btp * gm;
    }
    __syncthreads();
    // q = R[:n+1, :n] c2 (R_{p,k} vanishes for p > k + 1); each row's k range split over the two halves of
    // the workgroup as in the Gram pass below
    {
        const int half = tid / (WG / 2), pl = tid % (WG / 2);
        for (int p0 = 0; p0 <= n; p0 += WG / 2) {
            const int p = p0 + pl;
            double sq[4] = {0.0, 0.0, 0.0, 0.0};
            if (p <= n) {
                const int k0 = p > 0 ? p - 1 : 0;
                const int kmid = k0 + (n - k0) / 2;
                int k = half ? kmid : k0;
                const int ke = half ? n : kmid;
                for (; k + 3 < ke; k += 4) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) sq[i] += Rc[(int64_t)(k + i) * (nu + 1) + p] * c2[k + i];
                }
                for (; k < ke; ++k) sq[0] += Rc[(int64_t)k * (nu + 1) + p] * c2[k];
            }
            hsum[(int64_t)(half * (WG / 2) + pl) * 3] = (sq[0] + sq[1]) + (sq[2] + sq[3]);
            __syncthreads();
            if (half == 0 && p <= n) q[p] = hsum[(int64_t)pl * 3] + hsum[(int64_t)(WG / 2 + pl) * 3];
            __syncthreads();
        }
    }
    // one pass over the first n columns of G: G c1_prev, G c2 and G q. Thread (half, pl) takes column
    // p = p0 + pl and half of its k range (four running sums each, so that four loads of G are in flight);
    // the halves' sums meet in LDS and add in a fixed order.
    {
        const int half = tid / (WG / 2), pl = tid % (WG / 2);
        const int kmid = n / 2;
        const int kb = half ? kmid : 0, ke = half ? n : kmid;
        for (int p0 = 0; p0 < n; p0 += WG / 2) {
            const int p = p0 + pl;
            double sg[4] = {0.0, 0.0, 0.0, 0.0}, sv[4] = {0.0, 0.0, 0.0, 0.0}, sw[4] = {0.0, 0.0, 0.0, 0.0};
            if (p < n) {
                int k = kb;
                for (; k + 3 < ke; k += 4) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const double gkp = G[(int64_t)(k + i) * nu + p];
                        sg[i] += gkp * c1p[k + i];
                        sv[i] += gkp * c2[k + i];
                        sw[i] += gkp * q[k + i];
                    }
                }
                for (; k < ke; ++k) {
                    const double gkp = G[(int64_t)k * nu + p];
                    sg[0] += gkp * c1p[k];
                    sv[0] += gkp * c2[k];
                    sw[0] += gkp * q[k];
                }
            }
            double* hs = hsum + (int64_t)(half * (WG / 2) + pl) * 3;
            hs[0] = (sg[0] + sg[1]) + (sg[2] + sg[3]);
            hs[1] = (sv[0] + sv[1]) + (sv[2] + sv[3]);
            hs[2] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
            __syncthreads();
            if (half == 0 && p < n) {
                const double* h1 = hsum + (int64_t)(WG / 2 + pl) * 3;
                if (n >= 1) t[p] = (A[(int64_t)p * nu + (n - 1)] - (hs[0] + h1[0])) / btp;
                gc2[p] = hs[1] + h1[1];
                gq[p] = hs[2] + h1[2];
            }
            __syncthreads();
        }
    }
    __syncthreads();
    double p4 = 0.0, p5 = 0.0, p6 = 0.0;
    for (int p = tid; p < n; p += WG) {
        const double v = (t[p] - gc2[p]) / gm;
        G[(int64_t)p * nu + n] = v;
        G[(int64_t)n * nu + p] = v;
        p4 += c2[p] * t[p];
        p5 += c2[p] * gc2[p];
        p6 += v * q[p];
    }
    const double s_ct = bsum(p4), s_cgc = bsum(p5), s_vq = bsum(p6);
    const double gnn = (uu - 2.0 * s_ct + s_cgc) / gam2;
    if (tid == 0) G[(int64_t)n * nu + n] = gnn;
    const double En = (uty - s_ce) / gm;
    const double Fnn = (utsy - s_cg) / gm;
    for (int p = tid; p <= n; p += WG) {
        // (G q)_p over k <= n: the old columns, then column n (G[p][n] = G[n][p], just formed)
        const double sgq = p < n ? gq[p] + G[(int64_t)p * nu + n] * q[n] : s_vq + gnn * q[n];
        const double Ep = p < n ? e[p] : En;
        A[(int64_t)p * nu + n] = (Ep - sgq) / gm;
        const double Fp = p < n ? g[p] : Fnn;
        C1[(int64_t)b * nu + p] = (Fp - q[p]) / gm;
    }
    for (int k = tid; k < n; k += WG) {
        cA[(int64_t)k * B + b] = sc * c2[k];
        cB[(int64_t)k * B + b] = sc * g[k];
        if (cAf) {  // the same coefficients rounded once to the basis precision
            cAf[(int64_t)k * B + b] = (float)(sc * c2[k]);
            cBf[(int64_t)k * B + b] = (float)(sc * g[k]);
        }
    }
    if (tid == 0) {
        gam[b] = sc * gm;
        Fn[b] = sc * Fnn;
    }
}

LaunchInfo launch_coef(int B, int nu, int n, const double* red, double* A, double* G, double* R, double* C1,
                       double* BT, double* UU, double* cA, double* cB, float* cAf, float* cBf,
                       double* gam, double* Fn, int32_t* active, int32_t* nu_eff, double tau, const double* redb,
                       hipStream_t s) {
    const size_t lds = (size_t)(8 * (nu + 1) + 8 + 3 * WG) * sizeof(double);
    hipLaunchKernelGGL(k_coef, dim3(B), dim3(WG), lds, s, B, nu, n, red, A, G, R, C1, BT, UU, cA, cB, cAf, cBf, gam,
                       Fn, active, nu_eff, tau, redb);
    LaunchInfo li;
    li.wgs = B;
    const double nn = (double)n + 1.0;
    li.bytes = (double)B * (3.0 * nn * nn + 8.0 * nn) * 8.0;
    li.flops = (double)B * 8.0 * nn * nn;
    return li;
}

}  // namespace mar
