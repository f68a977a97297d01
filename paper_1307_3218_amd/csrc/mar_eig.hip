// Subspace eigensolve and Fermi-weighted assembly, one workgroup per seed.
//
// For seed j with m = nu_eff vectors, A = K^T H K (m x m, FP64) is reduced to
// tridiagonal form T = Q^T A Q by Householder reflections; the reflections are
// applied on the fly to the m x (1 + |P(j)|) matrix R = [e_1 | K[P(j), :]^T],
// so no m x m eigenvector matrix is ever formed. The implicit QL iteration
// with Wilkinson shifts then diagonalizes T, applying each plane rotation to
// the rows of R. At the end row alpha of R holds
//     R[alpha][0]     = y_1alpha            (first component of y_alpha)
//     R[alpha][1 + t] = e_i . v_alpha,  i = P(j)[t],  v_alpha = K y_alpha
// which is all the Green's-function assembly needs (Sec. 2):
//     rho_ij = 2 sum_alpha f_alpha (e_i.v_alpha)(e_j.v_alpha),
//     w_alpha = (e_j^T S v_alpha)(v_alpha^T e_j) = sqrt(S_jj) y_1alpha (e_j.v_alpha)
// (K^T S e_j = sqrt(S_jj) e_1 because u_1 = e_j / sqrt(S_jj) and K^T S K = I),
//     E_j = sum_{i in P(j)} rho_ij H_ij,   N_j = sum_{i in P(j)} rho_ij S_ij.
#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cstdint>

#include "mar_device.h"
#include "mar_internal.h"

namespace mar {

__device__ __forceinline__ double fermi_occ(double eps, double mu, double kT) {
    if (kT == 0.0) return eps < mu ? 1.0 : (eps > mu ? 0.0 : 0.5);
    const double x = (eps - mu) / kT;
    const double t = exp(-fabs(x));
    return x >= 0.0 ? t / (1.0 + t) : 1.0 / (1.0 + t);
}

// Logistic step F(x) = 1/(1+e^-x), and the window of a smoothed delta of width
// sigma over [a, b] (sigma = 0: sharp, 1/2 at an endpoint) for Eq. 3.
__device__ __forceinline__ double logistic_step(double x) {
    const double t = exp(-fabs(x));
    return x >= 0.0 ? 1.0 / (1.0 + t) : t / (1.0 + t);
}
__device__ __forceinline__ double smooth_step(double x, double sigma) {
    if (sigma == 0.0) return x > 0.0 ? 1.0 : (x < 0.0 ? 0.0 : 0.5);
    return logistic_step(x / sigma);
}
__device__ __forceinline__ double level_window(double eps, double a, double b, double sigma) {
    return smooth_step(b - eps, sigma) - smooth_step(a - eps, sigma);
}

// Sum over the 256 threads; every thread gets the same value (butterfly
// pairs add the same two operands, so all lanes agree bit for bit).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Lane t's double, read by the whole wavefront (t uniform).
__device__ __forceinline__ double lane_value(double x, int t) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)b, t);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), t);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Implicit QL with Wilkinson shifts on the symmetric tridiagonal (d, e),
// e[i] coupling d[i] and d[i+1], e[m-1] = 0 (Bowdler, Martin, Reinsch and
// Wilkinson's tql2 scheme). Run by one wavefront. The (d, e) recurrence is
// serial: every lane carries it with the same values. A sweep reads only the
// entries as they were when it began, so they are loaded 64 at a time into
// lane registers and broadcast with readlane, keeping LDS latency off the
// recurrence; the plane rotations are logged in cs/sn and then applied by the
// lanes to their columns l, l + 64, ... of R, carrying the row each rotation
// passes down. The split point is found by testing 64 subdiagonal entries at once.
// At most maxit iterations per eigenvalue; returns the number of eigenvalues
// left unconverged (0 on success).
__device__ int ql_implicit(double* d, double* e, int m, double* R, int nr, int lane, double* cs, double* sn,
                           int maxit) {
    int fails = 0;
    for (int l = 0; l < m; ++l) {
        int iter = 0;
        for (;;) {
            // first mm >= l with a negligible e[mm]; e[m-1] = 0 ends the search at m-1
            int mm = m - 1;
            for (int base = l; base < m - 1; base += 64) {
                const int t = base + lane;
                bool small = false;
                if (t < m - 1) small = fabs(e[t]) <= DBL_EPSILON * (fabs(d[t]) + fabs(d[t + 1]));
                const unsigned long long hit = __ballot(small);
                if (hit) {
                    mm = base + __ffsll(hit) - 1;
                    break;
                }
            }
            if (mm == l) break;
            if (++iter > maxit) {
                ++fails;
                break;
            }
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool split = false;
            int nrot = 0;
            double di1 = d[mm];   // d[i+1] as it was when the sweep began
            for (int i0 = mm - 1; i0 >= l && !split; i0 -= 64) {
                const int ii = i0 - lane;   // lane t holds e[i0-t], d[i0-t]
                const double eR = ii >= l ? e[ii] : 0.0, dR = ii >= l ? d[ii] : 0.0;
                const int nt = min(64, i0 - l + 1);
                // wait for these two loads here, so the loop below carries no LDS wait
                __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0), other counters unchanged
                for (int t = 0; t < nt; ++t) {
                    const int i = i0 - t;
                    const double ei = lane_value(eR, t), di = lane_value(dR, t);
                    const double f = s * ei, bb = c * ei, bb2 = 2.0 * bb;
                    const double ss = fma(f, f, g * g);
                    // r = sqrt(ss) and 1/(2r) by two coupled Goldschmidt steps from the reciprocal
                    // square root; tiny, huge or zero ss take the careful path below instead
                    const double y0 = __builtin_amdgcn_rsq(ss);
                    double gq = ss * y0, hq = 0.5 * y0;
                    double res = fma(-gq, hq, 0.5);
                    gq = fma(gq, res, gq);
                    hq = fma(hq, res, hq);
                    res = fma(-gq, hq, 0.5);
                    gq = fma(gq, res, gq);
                    hq = fma(hq, res, hq);
                    r = gq;
                    double rinv = 2.0 * hq;
                    if (!(ss > DBL_MIN && ss < DBL_MAX)) {
                        r = hypot(f, g);
                        rinv = r != 0.0 ? 1.0 / r : 0.0;
                        if (r == 0.0) {
                            e[i + 1] = r;
                            d[i + 1] = di1 - p;
                            e[mm] = 0.0;
                            split = true;
                            break;
                        }
                    }
                    e[i + 1] = r;
                    s = f * rinv;
                    c = g * rinv;
                    g = di1 - p;
                    r = (di - g) * s + c * bb2;   // c * (2 bb) equals (2 c) * bb exactly
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - bb;
                    cs[nrot] = c;
                    sn[nrot] = s;
                    ++nrot;
                    di1 = di;
                }
            }
            // rotation t acts on rows (mm-1-t, mm-t); row mm-t is final after it.
            // Four rotations at a time: their loads (rows not yet written) go out first.
            for (int col = lane; col < nr; col += 64) {
                double carry = R[mm * nr + col];
                int t = 0;
                for (; t + 4 <= nrot; t += 4) {
                    const int i = mm - 1 - t;
                    double a[4], cc[4], sv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        a[u] = R[(i - u) * nr + col];
                        cc[u] = cs[t + u];
                        sv[u] = sn[t + u];
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        R[(i - u + 1) * nr + col] = sv[u] * a[u] + cc[u] * carry;
                        carry = cc[u] * a[u] - sv[u] * carry;
                    }
                }
                for (; t < nrot; ++t) {
                    const int i = mm - 1 - t;
                    const double a0 = R[i * nr + col];
                    R[(i + 1) * nr + col] = sn[t] * a0 + cs[t] * carry;
                    carry = cs[t] * a0 - sn[t] * carry;
                }
                R[(mm - nrot) * nr + col] = carry;
            }
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
        }
    }
    return fails;
}

size_t eig_lds_bytes(int nu, int max_row, bool a_in_lds) {
    size_t n = (a_in_lds ? (size_t)nu * nu : 0) + (size_t)nu * (max_row + 1) + 4 * (size_t)nu + 8 + 72 + 64 + 2;
    return n * sizeof(double);
}

bool eig_a_fits_lds(int nu, int max_row) { return eig_lds_bytes(nu, max_row, true) <= 160 * 1024; }

// Rows K[P(j), :] of each seed, gathered from the seed-interleaved basis into
// Kp[(b * nu + k) * max_row + t] (FP64), with the seed's nu_eff copied beside
// them, so that the eigensolve can run while the basis is reused.
template <typename T>
__global__ __launch_bounds__(WG) void k_gather_rows(int nseeds, const int32_t* __restrict__ seeds, int B, int nu,
                                                    const int32_t* __restrict__ nu_eff_blk, const T* __restrict__ K,
                                                    int64_t stride, const int32_t* __restrict__ Hrp,
                                                    const int32_t* __restrict__ Hcol, int max_row,
                                                    double* __restrict__ Kp, int32_t* __restrict__ nu_copy) {
    const int b = blockIdx.x;
    if (b >= nseeds) return;
    const int m = nu_eff_blk[b];
    if (threadIdx.x == 0) nu_copy[b] = m;
    if (m <= 0) return;
    const int j = seeds[b];
    const int rlo = Hrp[j], nP = Hrp[j + 1] - rlo;
    for (int idx = threadIdx.x; idx < m * nP; idx += WG) {
        const int k = idx / nP, t = idx - k * nP;
        Kp[((int64_t)b * nu + k) * max_row + t] = (double)K[(int64_t)k * stride + (int64_t)Hcol[rlo + t] * B + b];
    }
}

template <bool LDS_A>
__global__ __launch_bounds__(WG) void k_eig(EigExtra ex, int nseeds, const int32_t* __restrict__ seeds, int nu,
                                            double* __restrict__ h, const int32_t* __restrict__ nu_eff_blk,
                                            const double* __restrict__ Kp, const int32_t* __restrict__ Hrp,
                                            const int32_t* __restrict__ Hcol, const double* __restrict__ Hval,
                                            const double* __restrict__ SvalH, const double* __restrict__ diagS,
                                            int max_row, double mu, double kT, double* __restrict__ rho,
                                            double* __restrict__ e_seed, double* __restrict__ n_seed,
                                            int32_t* __restrict__ nu_eff_out, double* __restrict__ eps_out,
                                            double* __restrict__ w_out, double* __restrict__ zc) {
    extern __shared__ double smem[];
    const int b = blockIdx.x;
    if (b >= nseeds) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = nu_eff_blk[b];
    double* eps_b = eps_out ? eps_out + (int64_t)b * nu : nullptr;
    double* w_b = w_out ? w_out + (int64_t)b * nu : nullptr;
    if (m <= 0) {
        if (tid == 0) {
            nu_eff_out[b] = m;
            e_seed[b] = 0.0;
            n_seed[b] = 0.0;
        }
        for (int a = tid; a < nu; a += WG) {
            if (eps_b) eps_b[a] = 0.0;
            if (w_b) w_b[a] = 0.0;
        }
        return;
    }
    const int j = seeds[b];
    const int rlo = Hrp[j];
    const int nP = Hrp[j + 1] - rlo;
    // columns of R: [e_1 | K[P(j),:]^T] (+ [K^T v_ref] in mode 2), or [e_1 | I_m] in mode 1
    const int NR = ex.mode == 1 ? m + 1 : (ex.mode == 2 ? nP + 2 : nP + 1);

    double* A;
    int ld;
    double* p = smem;
    if constexpr (LDS_A) {
        A = p;
        ld = m;
        p += (size_t)nu * nu;
    } else {
        A = h + (int64_t)b * nu * nu;
        ld = nu;
    }
    double* Rl = p;
    double* R = ex.mode == 1 ? ex.Rg + (int64_t)b * nu * (nu + 1) : Rl;
    p += (size_t)nu * (max_row + (ex.mode == 2 ? 2 : 1));
    double* d = p;
    p += nu;
    double* e = p;
    p += nu;
    double* v = p;
    p += nu;
    double* q = p;
    p += nu;
    double* red = p;
    p += 8;
    double* svec = ex.mode == 1 ? Rl : p;   // one value per column of R (mode 1: up to nu + 1, in R's unused LDS)
    p += 72;
    double* rhoL = p;
    p += 64;
    int* tjp = reinterpret_cast<int*>(p);

    // A = K^T H K from its computed upper triangle (h[b][k][n], k <= n), mirrored.
    const double* hb = h + (int64_t)b * nu * nu;
    if constexpr (LDS_A) {
        for (int r = wave; r < m; r += 4)
            for (int c = lane; c < m; c += 64) A[r * ld + c] = r <= c ? hb[(int64_t)r * nu + c] : hb[(int64_t)c * nu + r];
    } else {
        for (int r = wave; r < m; r += 4)
            for (int c = lane; c < r; c += 64) A[r * ld + c] = A[c * ld + r];
    }
    for (int idx = tid; idx < m * NR; idx += WG) {
        const int k = idx / NR, c = idx - k * NR;
        double r0;
        if (c == 0) r0 = k == 0 ? 1.0 : 0.0;
        else if (ex.mode == 1) r0 = k == c - 1 ? 1.0 : 0.0;
        else if (c <= nP) r0 = Kp[((int64_t)b * nu + k) * max_row + (c - 1)];
        else r0 = ex.pref[(int64_t)k * ex.pB + b];
        R[idx] = r0;
    }
    if (tid < nP && Hcol[rlo + tid] == j) *tjp = tid;
    __syncthreads();

    // Householder tridiagonalization, reflections also applied to R.
    for (int k = 0; k < m - 2; ++k) {
        const int len = m - k - 1;
        const double* xr = A + k * ld + k + 1;  // row k right of the diagonal = column k below it
        double part = 0.0;
        for (int i = 1 + tid; i < len; i += WG) part += xr[i] * xr[i];
        const double rest = block_sum(part, red);
        const double x0 = xr[0];
        if (rest == 0.0) {
            if (tid == 0) {
                d[k] = A[k * ld + k];
                e[k] = x0;
            }
            continue;
        }
        const double xx = rest + x0 * x0;
        const double alpha = -copysign(sqrt(xx), x0);
        const double vn = 1.0 / sqrt(2.0 * (xx - alpha * x0));
        for (int i = tid; i < len; i += WG) v[i] = (xr[i] - (i == 0 ? alpha : 0.0)) * vn;
        __syncthreads();
        // q = A22 v, then q = 2 (q - (v.q) v): A22 <- A22 - v q^T - q v^T
        double pv = 0.0;
        for (int i = tid; i < len; i += WG) {
            const double* col = A + (k + 1) * ld + (k + 1) + i;
            double s = 0.0;
            for (int jj = 0; jj < len; ++jj) s += col[jj * ld] * v[jj];
            q[i] = s;
            pv += s * v[i];
        }
        const double kp = block_sum(pv, red);
        for (int i = tid; i < len; i += WG) q[i] = 2.0 * (q[i] - kp * v[i]);
        __syncthreads();
        for (int r = wave; r < len; r += 4) {
            const double vr = v[r], qr = q[r];
            double* row = A + (k + 1 + r) * ld + (k + 1);
            for (int c = lane; c < len; c += 64) row[c] -= vr * q[c] + qr * v[c];
        }
        for (int cb = 0; cb < NR; cb += WG / 8) {
            const int c = cb + (tid >> 3), pi = tid & 7;
            double s = 0.0;
            if (c < NR)
                for (int i = pi; i < len; i += 8) s += v[i] * R[(k + 1 + i) * NR + c];
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            s += __shfl_xor(s, 4);
            if (c < NR && pi == 0) svec[c] = s;
        }
        __syncthreads();
        for (int idx = tid; idx < len * NR; idx += WG) {
            const int i = idx / NR, c = idx - i * NR;
            R[(k + 1 + i) * NR + c] -= 2.0 * v[i] * svec[c];
        }
        if (tid == 0) {
            d[k] = A[k * ld + k];
            e[k] = alpha;
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (m >= 2) {
            d[m - 2] = A[(m - 2) * ld + (m - 2)];
            e[m - 2] = A[(m - 2) * ld + (m - 1)];
            d[m - 1] = A[(m - 1) * ld + (m - 1)];
        } else {
            d[0] = A[0];
        }
        e[m - 1] = 0.0;
    }
    __syncthreads();
    // v, q are free after the reduction; R is in LDS except in mode 1 (a separate
    // call there, so that the LDS case compiles to LDS instructions)
    int* failp = tjp + 1;
    if (wave == 0) {
        int f;
        if (ex.mode == 1) f = ql_implicit(d, e, m, R, NR, lane, v, q, ex.ql_maxit);
        else f = ql_implicit(d, e, m, Rl, NR, lane, v, q, ex.ql_maxit);
        if (lane == 0) *failp = f;
    }
    __syncthreads();
    if (*failp != 0) {
        // an eigenvalue is still unconverged: the seed reports NU_NOCONV and NaN in every output
        const double nan = __builtin_nan("");
        if (ex.mode == 1) {
            for (int idx = tid; idx < m * m; idx += WG) {
                const int a = idx / m, c = idx - a * m;
                ex.Y[((int64_t)b * nu + a) * nu + c] = nan;
            }
        } else if (ex.mode == 2) {
            if (tid == 0) ex.phi[b] = nan;
        } else if (zc == nullptr) {
            for (int t = tid; t < nP; t += WG) rho[rlo + t] = nan;
            if (tid == 0) {
                e_seed[b] = nan;
                n_seed[b] = nan;
            }
        }
        for (int a = tid; a < nu; a += WG) {
            if (eps_b) eps_b[a] = nan;
            if (w_b) w_b[a] = nan;
        }
        if (tid == 0) nu_eff_out[b] = NU_NOCONV;
        return;
    }

    // Fermi-weighted assembly, or (zc != nullptr) keep the rows e_i.v_alpha,
    // i in P(j), for an assembly at a Fermi level found later (k_assemble).
    const int tj = *tjp;
    const double sq = sqrt(diagS[j]);
    if (ex.mode == 1) {   // the full subspace eigenvectors y_alpha and levels
        for (int idx = tid; idx < m * m; idx += WG) {
            const int a = idx / m, c = idx - a * m;
            ex.Y[((int64_t)b * nu + a) * nu + c] = R[a * NR + 1 + c];
        }
        for (int a = tid; a < nu; a += WG) eps_b[a] = a < m ? d[a] : 0.0;
        if (tid == 0) nu_eff_out[b] = m;
        return;
    }
    if (ex.mode == 2) {   // Eq. 3 with the inner-product signs: sum_alpha s_alpha (e_j.v_alpha) window_alpha
        if (tid == 0) {
            const double lo = ex.win[1], hi = ex.win[2];
            double phi = 0.0;
            for (int a = 0; a < m; ++a) {
                const double c = R[a * NR + 1 + tj] * level_window(d[a], lo, hi, ex.sigma);
                phi += R[a * NR + NR - 1] >= 0.0 ? c : -c;
            }
            ex.phi[b] = phi;
            nu_eff_out[b] = m;
        }
        return;
    }
    if (zc != nullptr) {
        double* zb = zc + (int64_t)b * nu * max_row;
        for (int idx = tid; idx < m * nP; idx += WG) {
            const int a = idx / nP, t = idx - a * nP;
            zb[a * max_row + t] = R[a * NR + 1 + t];
        }
        for (int a = tid; a < m; a += WG) {
            eps_b[a] = d[a];
            w_b[a] = sq * R[a * NR] * R[a * NR + 1 + tj];
        }
        for (int a = m + tid; a < nu; a += WG) {
            eps_b[a] = 0.0;
            w_b[a] = 0.0;
        }
        if (tid == 0) nu_eff_out[b] = m;
        return;
    }
    double* fz = q;
    for (int a = tid; a < m; a += WG) {
        const double ea = d[a];
        const double zj = R[a * NR + 1 + tj];
        fz[a] = fermi_occ(ea, mu, kT) * zj;
        if (eps_b) eps_b[a] = ea;
        if (w_b) w_b[a] = sq * R[a * NR] * zj;
    }
    for (int a = m + tid; a < nu; a += WG) {
        if (eps_b) eps_b[a] = 0.0;
        if (w_b) w_b[a] = 0.0;
    }
    __syncthreads();
    for (int cb = 0; cb < nP; cb += WG / 8) {
        const int t = cb + (tid >> 3), pi = tid & 7;
        double s = 0.0;
        if (t < nP)
            for (int a = pi; a < m; a += 8) s += fz[a] * R[a * NR + 1 + t];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        if (t < nP && pi == 0) {
            const double r = 2.0 * s;
            rho[rlo + t] = r;
            rhoL[t] = r;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double E = 0.0, N = 0.0;
        for (int t = 0; t < nP; ++t) {
            E += rhoL[t] * Hval[rlo + t];
            N += rhoL[t] * SvalH[rlo + t];
        }
        e_seed[b] = E;
        n_seed[b] = N;
        nu_eff_out[b] = m;
    }
}

// Lets kernel f use up to 160 KB of dynamic LDS. The attribute belongs to the current device, so it is
// set once per device (bit d of done for device d; concurrent first calls both set it, which is harmless).
static void allow_full_lds(const void* f, std::atomic<uint64_t>& done) {
    int dev = 0;
    const bool known = hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64;
    const uint64_t bit = known ? 1ull << dev : 0;
    if (known && (done.load(std::memory_order_acquire) & bit)) return;
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (known) done.fetch_or(bit, std::memory_order_acq_rel);
}

LaunchInfo launch_eig(int nseeds, const int32_t* seeds, int nu, double* h, const int32_t* nu_eff_blk,
                      const double* Kp, const int32_t* Hrp, const int32_t* Hcol, const double* Hval,
                      const double* SvalH, const double* diagS, int max_row, double mu, double kT, double* rho,
                      double* e_seed, double* n_seed, int32_t* nu_eff_out, double* eps_out, double* w_out,
                      double* zc, const EigExtra& ex, hipStream_t s) {
    const int rcols = max_row + (ex.mode == 2 ? 1 : 0);   // R's LDS share (mode 1 keeps R in global memory)
    const bool lds_a = eig_a_fits_lds(nu, rcols);
    const size_t lds = eig_lds_bytes(nu, rcols, lds_a);
    if (lds_a) {
        static std::atomic<uint64_t> done{0};
        allow_full_lds((const void*)k_eig<true>, done);
        hipLaunchKernelGGL((k_eig<true>), dim3(nseeds), dim3(WG), lds, s, ex, nseeds, seeds, nu, h, nu_eff_blk, Kp, Hrp,
                           Hcol, Hval, SvalH, diagS, max_row, mu, kT, rho, e_seed, n_seed, nu_eff_out, eps_out, w_out,
                           zc);
    } else {
        static std::atomic<uint64_t> done{0};
        allow_full_lds((const void*)k_eig<false>, done);
        hipLaunchKernelGGL((k_eig<false>), dim3(nseeds), dim3(WG), lds, s, ex, nseeds, seeds, nu, h, nu_eff_blk, Kp,
                           Hrp, Hcol, Hval, SvalH, diagS, max_row, mu, kT, rho, e_seed, n_seed, nu_eff_out, eps_out,
                           w_out, zc);
    }
    LaunchInfo li;
    li.wgs = nseeds;
    const double nv = (double)nu;
    li.bytes = (double)nseeds * (nv * nv * 8.0 + nv * max_row * 8.0 + (max_row + 3) * 8.0 * 3);
    li.flops = (double)nseeds * ((4.0 / 3.0) * nv * nv * nv + 4.0 * nv * nv * (max_row + 1));
    return li;
}

// ---------------------------------------------------------------------------
// Assembly at a Fermi level held on the device (after k_eig with zc != nullptr):
// the same sums, in the same order, as the fused epilogue of k_eig.
__global__ __launch_bounds__(WG) void k_assemble(int nseeds, const int32_t* __restrict__ seeds, int nu,
                                                 const int32_t* __restrict__ nu_eff, const double* __restrict__ eps,
                                                 const double* __restrict__ zc, int max_row,
                                                 const int32_t* __restrict__ Hrp, const int32_t* __restrict__ Hcol,
                                                 const double* __restrict__ Hval, const double* __restrict__ SvalH,
                                                 const double* __restrict__ mu_p, double kT, double* __restrict__ rho,
                                                 double* __restrict__ e_seed, double* __restrict__ n_seed) {
    __shared__ double fz[MAX_NU_ASSEMBLE];
    __shared__ double rhoL[64];
    __shared__ int tjs;
    const int b = blockIdx.x, tid = threadIdx.x;
    if (b >= nseeds) return;
    const int m = nu_eff[b];
    if (m <= 0) {
        // a seed whose subspace eigensolve did not converge gets NaN outputs, as in k_eig
        const double fill = m == NU_NOCONV ? __builtin_nan("") : 0.0;
        if (m == NU_NOCONV)
            for (int t = Hrp[seeds[b]] + tid; t < Hrp[seeds[b] + 1]; t += WG) rho[t] = fill;
        if (tid == 0) {
            e_seed[b] = fill;
            n_seed[b] = fill;
        }
        return;
    }
    const int j = seeds[b];
    const int rlo = Hrp[j], nP = Hrp[j + 1] - rlo;
    if (tid < nP && Hcol[rlo + tid] == j) tjs = tid;
    __syncthreads();
    const int tj = tjs;
    const double mu = *mu_p;
    const double* zb = zc + (int64_t)b * nu * max_row;
    for (int a = tid; a < m; a += WG) fz[a] = fermi_occ(eps[(int64_t)b * nu + a], mu, kT) * zb[a * max_row + tj];
    __syncthreads();
    for (int cb = 0; cb < nP; cb += WG / 8) {
        const int t = cb + (tid >> 3), pi = tid & 7;
        double s = 0.0;
        if (t < nP)
            for (int a = pi; a < m; a += 8) s += fz[a] * zb[a * max_row + t];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        if (t < nP && pi == 0) {
            const double r = 2.0 * s;
            rho[rlo + t] = r;
            rhoL[t] = r;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double E = 0.0, N = 0.0;
        for (int t = 0; t < nP; ++t) {
            E += rhoL[t] * Hval[rlo + t];
            N += rhoL[t] * SvalH[rlo + t];
        }
        e_seed[b] = E;
        n_seed[b] = N;
    }
}

LaunchInfo launch_assemble(int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff, const double* eps,
                           const double* zc, int max_row, const int32_t* Hrp, const int32_t* Hcol,
                           const double* Hval, const double* SvalH, const double* mu, double kT, double* rho,
                           double* e_seed, double* n_seed, hipStream_t s) {
    LaunchInfo li;
    if (nu > MAX_NU_ASSEMBLE || max_row > 64) {
        li.wgs = -1;
        return li;
    }
    if (nseeds > 0)
        hipLaunchKernelGGL(k_assemble, dim3(nseeds), dim3(WG), 0, s, nseeds, seeds, nu, nu_eff, eps, zc, max_row, Hrp,
                           Hcol, Hval, SvalH, mu, kT, rho, e_seed, n_seed);
    li.wgs = nseeds;
    li.bytes = (double)nseeds * ((double)nu * (max_row + 1) * 8.0 + 3.0 * max_row * 8.0);
    li.flops = (double)nseeds * 2.0 * nu * (max_row + 1);
    return li;
}

// ---------------------------------------------------------------------------
// Fermi level on the device: mu with N(mu) = sum_j 2 sum_alpha f((eps_alpha^(j)
// - mu)/kT) w_alpha^(j) equal to n_target, by bisection on [min eps - 40 kT,
// max eps + 40 kT] over the listed seeds' subspace levels (alpha < nu_eff).
// st = {lo, hi, mu}. Every sum runs in a fixed order.
constexpr int MU_WGS = 512;   // workgroups of the counting kernel

__device__ __forceinline__ void wg_minmax(double& lo, double& hi, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off));
        hi = fmax(hi, __shfl_xor(hi, off));
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red[wave] = lo;
        red[4 + wave] = hi;
    }
    __syncthreads();
    lo = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
    hi = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
}

__global__ __launch_bounds__(WG) void k_mu_bounds(int64_t nseeds, int nu, const int32_t* __restrict__ nu_eff,
                                                  const double* __restrict__ eps, double* __restrict__ part) {
    __shared__ double red[8];
    double lo = INFINITY, hi = -INFINITY;
    const int64_t npair = nseeds * nu;
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < npair; p += (int64_t)gridDim.x * WG) {
        const int64_t b = p / nu;
        const int a = (int)(p - b * nu);
        if (a < nu_eff[b]) {
            lo = fmin(lo, eps[p]);
            hi = fmax(hi, eps[p]);
        }
    }
    wg_minmax(lo, hi, red);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = lo;
        part[2 * blockIdx.x + 1] = hi;
    }
}

__global__ __launch_bounds__(64) void k_mu_init(int nwg, const double* __restrict__ part, double kT,
                                                double* __restrict__ st) {
    if (threadIdx.x != 0) return;
    double lo = INFINITY, hi = -INFINITY;
    for (int g = 0; g < nwg; ++g) {
        lo = fmin(lo, part[2 * g]);
        hi = fmax(hi, part[2 * g + 1]);
    }
    if (!(lo <= hi)) lo = hi = 0.0;   // no levels at all
    st[0] = lo - 40.0 * kT;
    st[1] = hi + 40.0 * kT;
    st[2] = 0.5 * (st[0] + st[1]);
}

__global__ __launch_bounds__(WG) void k_mu_count(int64_t nseeds, int nu, const int32_t* __restrict__ nu_eff,
                                                 const double* __restrict__ eps, const double* __restrict__ w,
                                                 double kT, const double* __restrict__ st, double* __restrict__ part) {
    __shared__ double red[8];
    const double mid = 0.5 * (st[0] + st[1]);
    double s = 0.0;
    const int64_t npair = nseeds * nu;
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < npair; p += (int64_t)gridDim.x * WG) {
        const int64_t b = p / nu;
        const int a = (int)(p - b * nu);
        if (a < nu_eff[b]) s += 2.0 * fermi_occ(eps[p], mid, kT) * w[p];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(64) void k_mu_step(int nwg, const double* __restrict__ part, double n_target,
                                                double* __restrict__ st, int last, double* __restrict__ mu_out) {
    if (threadIdx.x != 0) return;
    double n = 0.0;
    for (int g = 0; g < nwg; ++g) n += part[g];
    const double mid = 0.5 * (st[0] + st[1]);
    if (n < n_target) st[0] = mid;
    else st[1] = mid;
    if (last) {
        st[2] = 0.5 * (st[0] + st[1]);
        if (mu_out) *mu_out = st[2];
    }
}

LaunchInfo launch_fermi_search(int64_t nseeds, int nu, const int32_t* nu_eff, const double* eps, const double* w,
                               double n_target, double kT, int iters, double* part, double* st, double* mu_out,
                               hipStream_t s) {
    const int64_t npair = nseeds * nu;
    int nwg = (int)std::min<int64_t>(MU_WGS, std::max<int64_t>(1, (npair + WG - 1) / WG));
    hipLaunchKernelGGL(k_mu_bounds, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, part);
    hipLaunchKernelGGL(k_mu_init, dim3(1), dim3(64), 0, s, nwg, part, kT, st);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_mu_count, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, w, kT, st, part);
        hipLaunchKernelGGL(k_mu_step, dim3(1), dim3(64), 0, s, nwg, part, n_target, st, it + 1 == iters ? 1 : 0,
                           mu_out);
    }
    LaunchInfo li;
    li.wgs = nwg;
    li.bytes = (double)(iters + 1) * npair * 20.0;
    li.flops = (double)iters * npair * 30.0;
    return li;
}

// ---------------------------------------------------------------------------
// Eigen states (Sec. 3, Eq. 3; Appendix): integrated density of states
//   n(eta) = sum_j sum_alpha w_alpha^(j) F((eta - eps_alpha^(j)) / sigma)
// (F the logistic step; sigma = 0: the unit step, 1/2 at 0), bisected for the
// three counts k - 1, k - 1/2 and k at once on [min eps - 1, max eps + 1].
// st = {lo, hi} x 3; lv = {eta(k - 1/2), eta(k - 1), eta(k)}.
__global__ __launch_bounds__(64) void k_dos_init(int nwg, const double* __restrict__ part, double* __restrict__ st) {
    if (threadIdx.x != 0) return;
    double lo = INFINITY, hi = -INFINITY;
    for (int g = 0; g < nwg; ++g) {
        lo = fmin(lo, part[2 * g]);
        hi = fmax(hi, part[2 * g + 1]);
    }
    if (!(lo <= hi)) lo = hi = 0.0;
    for (int t = 0; t < 3; ++t) {
        st[2 * t] = lo - 1.0;
        st[2 * t + 1] = hi + 1.0;
    }
}

__global__ __launch_bounds__(WG) void k_dos_count(int64_t nseeds, int nu, const int32_t* __restrict__ nu_eff,
                                                  const double* __restrict__ eps, const double* __restrict__ w,
                                                  double sigma, const double* __restrict__ st,
                                                  double* __restrict__ part) {
    __shared__ double red[8];
    double mid[3], c[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < 3; ++t) mid[t] = 0.5 * (st[2 * t] + st[2 * t + 1]);
    const int64_t npair = nseeds * nu;
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < npair; p += (int64_t)gridDim.x * WG) {
        const int64_t b = p / nu;
        const int a = (int)(p - b * nu);
        if (a < nu_eff[b]) {
#pragma unroll
            for (int t = 0; t < 3; ++t) c[t] += w[p] * smooth_step(mid[t] - eps[p], sigma);
        }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const double v = block_sum(c[t], red);
        if (threadIdx.x == 0) part[3 * blockIdx.x + t] = v;
    }
}

__global__ __launch_bounds__(64) void k_dos_step(int nwg, const double* __restrict__ part, int k,
                                                 double* __restrict__ st, int last, double* __restrict__ lv) {
    if (threadIdx.x != 0) return;
    const double target[3] = {k - 1.0, k - 0.5, (double)k};
    for (int t = 0; t < 3; ++t) {
        double n = 0.0;
        for (int g = 0; g < nwg; ++g) n += part[3 * g + t];
        const double mid = 0.5 * (st[2 * t] + st[2 * t + 1]);
        if (n < target[t]) st[2 * t] = mid;
        else st[2 * t + 1] = mid;
    }
    if (last) {
        lv[0] = 0.5 * (st[2] + st[3]);   // eps_k = eta(k - 1/2)
        lv[1] = 0.5 * (st[0] + st[1]);   // eta(k - 1)
        lv[2] = 0.5 * (st[4] + st[5]);   // eta(k)
    }
}

LaunchInfo launch_dos_search(int64_t nseeds, int nu, const int32_t* nu_eff, const double* eps, const double* w,
                             double sigma, int k, int iters, double* part, double* st, double* lv, hipStream_t s) {
    const int64_t npair = nseeds * nu;
    const int nwg = (int)std::min<int64_t>(MU_WGS, std::max<int64_t>(1, (npair + WG - 1) / WG));
    hipLaunchKernelGGL(k_mu_bounds, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, part);
    hipLaunchKernelGGL(k_dos_init, dim3(1), dim3(64), 0, s, nwg, part, st);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_dos_count, dim3(nwg), dim3(WG), 0, s, nseeds, nu, nu_eff, eps, w, sigma, st, part);
        hipLaunchKernelGGL(k_dos_step, dim3(1), dim3(64), 0, s, nwg, part, k, st, it + 1 == iters ? 1 : 0, lv);
    }
    LaunchInfo li;
    li.wgs = nwg;
    li.bytes = (double)(iters + 1) * npair * 20.0;
    li.flops = (double)iters * npair * 90.0;
    return li;
}

// Contributions c_alpha^(j) = (e_j . v_alpha^(j)) window_alpha of every seed
// (kept rows zc, levels eps) and the reference: the largest |c| (first seed,
// then first alpha, on ties). ref = {position b, alpha, seed j}; refseed[0] = j.
__global__ __launch_bounds__(WG) void k_es_contrib(int nseeds, const int32_t* __restrict__ seeds, int nu,
                                                   const int32_t* __restrict__ nu_eff, const double* __restrict__ eps,
                                                   const double* __restrict__ zc, int max_row,
                                                   const int32_t* __restrict__ Hrp, const int32_t* __restrict__ Hcol,
                                                   const double* __restrict__ lv, double sigma,
                                                   double* __restrict__ cmax, int32_t* __restrict__ amax) {
    __shared__ int tjs;
    const int b = blockIdx.x;
    if (b >= nseeds) return;
    const int m = nu_eff[b];
    if (m <= 0) {
        if (threadIdx.x == 0) {
            cmax[b] = -1.0;
            amax[b] = 0;
        }
        return;
    }
    const int j = seeds[b];
    const int rlo = Hrp[j], nP = Hrp[j + 1] - rlo;
    if ((int)threadIdx.x < nP && Hcol[rlo + threadIdx.x] == j) tjs = threadIdx.x;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double* zb = zc + (int64_t)b * nu * max_row;
    double best = -1.0;
    int ba = 0;
    for (int a = 0; a < m; ++a) {
        const double c = fabs(zb[a * max_row + tjs] * level_window(eps[(int64_t)b * nu + a], lv[1], lv[2], sigma));
        if (c > best) {
            best = c;
            ba = a;
        }
    }
    cmax[b] = best;
    amax[b] = ba;
}

__global__ __launch_bounds__(64) void k_es_argmax(int nseeds, const int32_t* __restrict__ seeds,
                                                  const double* __restrict__ cmax, const int32_t* __restrict__ amax,
                                                  int32_t* __restrict__ ref, int32_t* __restrict__ refseed) {
    if (threadIdx.x != 0) return;
    double best = -1.0;
    int bb = 0;
    for (int b = 0; b < nseeds; ++b)
        if (cmax[b] > best) {
            best = cmax[b];
            bb = b;
        }
    ref[0] = bb;
    ref[1] = nseeds > 0 ? amax[bb] : 0;
    ref[2] = nseeds > 0 ? seeds[bb] : 0;
    refseed[0] = ref[2];
}

LaunchInfo launch_es_reference(int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff, const double* eps,
                               const double* zc, int max_row, const int32_t* Hrp, const int32_t* Hcol,
                               const double* lv, double sigma, double* cmax, int32_t* amax, int32_t* ref,
                               int32_t* refseed, hipStream_t s) {
    if (nseeds > 0)
        hipLaunchKernelGGL(k_es_contrib, dim3(nseeds), dim3(WG), 0, s, nseeds, seeds, nu, nu_eff, eps, zc, max_row, Hrp,
                           Hcol, lv, sigma, cmax, amax);
    hipLaunchKernelGGL(k_es_argmax, dim3(1), dim3(64), 0, s, nseeds, seeds, cmax, amax, ref, refseed);
    LaunchInfo li;
    li.wgs = nseeds;
    li.bytes = (double)nseeds * nu * 16.0;
    return li;
}

// Reference seed (solved alone, B = 1): pick among its subspace eigenvectors
// the one with the largest |(e_j . v_alpha) window_alpha| (v_alpha = K y_alpha),
// and form v_ref = K y_ref over all rows.
template <typename T>
__global__ __launch_bounds__(WG) void k_es_pick(const T* __restrict__ K, int64_t stride, const int32_t* __restrict__ seed,
                                                int nu, const int32_t* __restrict__ nu_eff,
                                                const double* __restrict__ Y, const double* __restrict__ eps,
                                                const double* __restrict__ lv, double sigma,
                                                double* __restrict__ yref) {
    __shared__ double cs[WG];
    __shared__ int as[WG];
    const int m = nu_eff[0];
    const int j = seed[0];
    double best = -1.0;
    int ba = 0;
    for (int a = threadIdx.x; a < m; a += WG) {
        double z = 0.0;
        for (int k = 0; k < m; ++k) z += (double)K[(int64_t)k * stride + j] * Y[(int64_t)a * nu + k];
        const double c = fabs(z * level_window(eps[a], lv[1], lv[2], sigma));
        if (c > best) {
            best = c;
            ba = a;
        }
    }
    cs[threadIdx.x] = best;
    as[threadIdx.x] = ba;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int t = 1; t < WG; ++t)
        if (cs[t] > best || (cs[t] == best && as[t] < ba)) {
            best = cs[t];
            ba = as[t];
        }
    for (int k = 0; k < nu; ++k) yref[k] = k < m ? Y[(int64_t)ba * nu + k] : 0.0;
}

template <typename T>
__global__ __launch_bounds__(WG) void k_es_vref(const T* __restrict__ K, int64_t stride, int64_t M, int nu,
                                                const int32_t* __restrict__ nu_eff, const double* __restrict__ yref,
                                                double* __restrict__ vref) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= M) return;
    const int m = nu_eff[0];
    double v = 0.0;
    for (int k = 0; k < m; ++k) v += (double)K[(int64_t)k * stride + i] * yref[k];
    vref[i] = v;
}

template <typename T>
LaunchInfo launch_es_refvec(const T* K, int64_t stride, int64_t M, const int32_t* seed, int nu,
                            const int32_t* nu_eff, const double* Y, const double* eps, const double* lv, double sigma,
                            double* yref, double* vref, hipStream_t s) {
    hipLaunchKernelGGL((k_es_pick<T>), dim3(1), dim3(WG), 0, s, K, stride, seed, nu, nu_eff, Y, eps, lv, sigma, yref);
    const int64_t wgs = (M + WG - 1) / WG;
    hipLaunchKernelGGL((k_es_vref<T>), dim3((unsigned)wgs), dim3(WG), 0, s, K, stride, M, nu, nu_eff, yref, vref);
    LaunchInfo li;
    li.wgs = wgs;
    li.bytes = (double)nu * M * (sizeof(T) + 8.0 / nu);
    return li;
}
template LaunchInfo launch_es_refvec<float>(const float*, int64_t, int64_t, const int32_t*, int, const int32_t*,
                                            const double*, const double*, const double*, double, double*, double*,
                                            hipStream_t);
template LaunchInfo launch_es_refvec<double>(const double*, int64_t, int64_t, const int32_t*, int, const int32_t*,
                                             const double*, const double*, const double*, double, double*, double*,
                                             hipStream_t);

template <typename T>
static LaunchInfo launch_gather_t(int B, int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff_blk,
                                  const T* K, int64_t stride, const int32_t* Hrp, const int32_t* Hcol, int max_row,
                                  double* Kp, int32_t* nu_copy, hipStream_t s) {
    hipLaunchKernelGGL((k_gather_rows<T>), dim3(nseeds), dim3(WG), 0, s, nseeds, seeds, B, nu, nu_eff_blk, K, stride, Hrp,
                       Hcol, max_row, Kp, nu_copy);
    LaunchInfo li;
    li.wgs = nseeds;
    li.bytes = (double)nseeds * nu * max_row * (sizeof(T) + 8.0);
    return li;
}

template <>
LaunchInfo launch_gather<float>(int B, int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff_blk,
                                const float* K, int64_t stride, const int32_t* Hrp, const int32_t* Hcol, int max_row,
                                double* Kp, int32_t* nu_copy, hipStream_t s) {
    return launch_gather_t<float>(B, nseeds, seeds, nu, nu_eff_blk, K, stride, Hrp, Hcol, max_row, Kp, nu_copy, s);
}

template <>
LaunchInfo launch_gather<double>(int B, int nseeds, const int32_t* seeds, int nu, const int32_t* nu_eff_blk,
                                 const double* K, int64_t stride, const int32_t* Hrp, const int32_t* Hcol, int max_row,
                                 double* Kp, int32_t* nu_copy, hipStream_t s) {
    return launch_gather_t<double>(B, nseeds, seeds, nu, nu_eff_blk, K, stride, Hrp, Hcol, max_row, Kp, nu_copy, s);
}

}  // namespace mar
