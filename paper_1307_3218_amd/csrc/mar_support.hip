// Support of the Krylov vectors of one seed block, and the work plan of the
// projection sweep restricted to it.
//
// The basis vector u_k of seed j (k = 0, 1, ...; u_0 = e_j / sqrt(S_jj)) is
// formed from e_j by k products with H and S and combinations with earlier
// basis vectors (Sec. 2, the Krylov subspace of Eq. 1 with b = e_j), and S's
// pattern lies inside H's. So u_k vanishes on every row more than k hops from
// j in the graph of H's pattern, and so do the unnormalized residual written
// into slab k and every partial result built from slabs <= k.
//
// For a block of seeds, dist(I) is the smallest hop count from the block row
// of any seed of the block to block row I (BFS over H's 4x4 block pattern).
// A row tile is 4 * WG 16-byte vectors of a slab, i.e. WG / P block rows; its
// distance D(t) is the smallest dist of its block rows. Slab k of the block is
// exactly zero on every tile with D(t) > k, and the streaming kernels skip
// those tiles: the values they produce are those of the full sweep, up to the
// order of the partial sums. Distances above hmax are stored as SUP_FAR.
//
// The tile list holds the tiles with D <= hmax sorted by (D, tile index);
// cnt[h] is the number of tiles with D <= h, so the tiles on which slab k can
// be nonzero are the first cnt[k] list entries.
#include "mar_device.h"
#include "mar_internal.h"

namespace mar {

__global__ __launch_bounds__(WG) void k_sup_fill(int32_t* __restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) d[i] = SUP_FAR;
}

__global__ __launch_bounds__(WG) void k_sup_seed(const int32_t* __restrict__ seeds, int ns, int64_t M,
                                                 int32_t* __restrict__ dist) {
    const int b = blockIdx.x * WG + threadIdx.x;
    if (b < ns) {
        const int j = seeds[b];
        if (j >= 0 && j < M) dist[j / 4] = 0;
    }
}

// One BFS level: a block row not yet reached gets h when a block column of its
// row was reached at h - 1. Rows written in this launch hold h, never h - 1,
// so the in-place update reads only finished levels.
__global__ __launch_bounds__(WG) void k_sup_hop(int64_t nbrow, const int32_t* __restrict__ brp,
                                                const int32_t* __restrict__ bcol, int32_t* dist, int h) {
    const int64_t I = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (I >= nbrow || dist[I] != SUP_FAR) return;
    const int lo = brp[I], hi = brp[I + 1];
    for (int p = lo; p < hi; ++p)
        if (dist[bcol[p]] == h - 1) {
            dist[I] = h;
            return;
        }
}

__global__ __launch_bounds__(WG) void k_sup_tiles(int64_t nbrow, int bpt, int64_t ntiles,
                                                  const int32_t* __restrict__ dist, int hmax,
                                                  int32_t* __restrict__ D) {
    const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= ntiles) return;
    const int64_t I0 = t * bpt, I1 = I0 + bpt < nbrow ? I0 + bpt : nbrow;
    int m = SUP_FAR;
    for (int64_t I = I0; I < I1; ++I) m = min(m, dist[I]);
    D[t] = m <= hmax ? m : SUP_FAR;
}

// cnt[h] = number of tiles with D <= h; one workgroup per h.
__global__ __launch_bounds__(WG) void k_sup_count(int64_t ntiles, const int32_t* __restrict__ D,
                                                  int32_t* __restrict__ cnt) {
    const int h = blockIdx.x;
    int c = 0;
    for (int64_t t = threadIdx.x; t < ntiles; t += WG) c += D[t] <= h ? 1 : 0;
    __shared__ int s[WG];
    s[threadIdx.x] = c;
    __syncthreads();
    for (int w = WG / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[h] = s[0];
}

// Tiles with D == h, in index order, into list positions cnt[h-1] ...; one
// workgroup per h (stable compaction by wavefront ballots).
__global__ __launch_bounds__(WG) void k_sup_scatter(int64_t ntiles, const int32_t* __restrict__ D,
                                                    const int32_t* __restrict__ cnt, int32_t* __restrict__ list,
                                                    int32_t* __restrict__ Dl) {
    constexpr int NW = WG / 64;
    const int h = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __shared__ int wsum[NW];
    int64_t pos = h > 0 ? cnt[h - 1] : 0;
    for (int64_t base = 0; base < ntiles; base += WG) {
        const int64_t t = base + threadIdx.x;
        const bool f = t < ntiles && D[t] == h;
        const unsigned long long m = __ballot(f);
        const int before = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wv] = __popcll(m);
        __syncthreads();
        int woff = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            woff += i < wv ? wsum[i] : 0;
            tot += wsum[i];
        }
        if (f) {
            list[pos + woff + before] = (int32_t)t;
            Dl[pos + woff + before] = h;
        }
        pos += tot;
        __syncthreads();
    }
}

LaunchInfo launch_support(int64_t M, int64_t nbrow, const int32_t* brp, const int32_t* bcol, int64_t nnzb,
                          const int32_t* seeds, int ns, int bpt, int hmax, int hcnt, int32_t* dist, int32_t* D,
                          int32_t* cnt, int32_t* list, int32_t* Dl, hipStream_t s) {
    const int64_t ntiles = (nbrow + bpt - 1) / bpt;
    const unsigned rw = (unsigned)((nbrow + WG - 1) / WG), tw = (unsigned)((ntiles + WG - 1) / WG);
    hipLaunchKernelGGL(k_sup_fill, dim3(rw), dim3(WG), 0, s, dist, nbrow);
    if (ns > 0) hipLaunchKernelGGL(k_sup_seed, dim3((ns + WG - 1) / WG), dim3(WG), 0, s, seeds, ns, M, dist);
    for (int h = 1; h <= hmax; ++h) hipLaunchKernelGGL(k_sup_hop, dim3(rw), dim3(WG), 0, s, nbrow, brp, bcol, dist, h);
    hipLaunchKernelGGL(k_sup_tiles, dim3(tw), dim3(WG), 0, s, nbrow, bpt, ntiles, dist, hmax, D);
    hipLaunchKernelGGL(k_sup_count, dim3(hcnt + 1), dim3(WG), 0, s, ntiles, D, cnt);
    hipLaunchKernelGGL(k_sup_scatter, dim3(hmax + 1), dim3(WG), 0, s, ntiles, D, cnt, list, Dl);
    LaunchInfo li;
    li.wgs = rw;
    li.bytes = (double)hmax * ((double)nbrow * 8.0 + (double)nnzb * 4.0) + 2.0 * (hmax + 1) * (double)ntiles * 4.0;
    return li;
}

// Work plan of the projection sweep of step n (nk = n + 1 slabs in chunks of
// kg): chunk ks reads the tiles on which one of its slabs can be nonzero, the
// first cnt[min(ks*kg + kg - 1, n)] list entries. The list is cut into groups
// of Tg consecutive entries, Tg >= ceil(W / G) for W tile-chunk pairs in all,
// so that at most G workgroups (at most one per chunk and group when G is
// smaller than the chunks) share the work evenly. Group g needs the chunks
// from ksmin(g) = D(first entry) / kg on; its chunks get consecutive
// workgroup numbers (off[g] + ks - ksmin(g)), so the workgroups that re-read
// a group's right-hand-side tiles run side by side. Layout of plan (int32):
//   [0] groups, [1] Tg, [2] workgroups used, [3] chunks; [8, 8 + grid) off;
//   then ksmin [grid], then the (group, chunk) of each workgroup, [grid] each
//   (group -1: idle). The number of workgroups used never exceeds G + chunks.
// Workgroup i writes the plan of step n0 + i at plans + i * pstride (the counts
// are fixed once the block's search is done, so every step's plan is made at once).
__global__ __launch_bounds__(WG) void k_projr_plan(const int32_t* __restrict__ cnt, const int32_t* __restrict__ Dl,
                                                   int n0, int kg, int64_t G, int64_t pstride,
                                                   int32_t* __restrict__ plans) {
    const int tid = threadIdx.x;
    const int n = n0 + (int)blockIdx.x;
    const int64_t grid = projr_sp_grid(G, n + 1, kg);
    int32_t* plan = plans + (int64_t)blockIdx.x * pstride;
    const int nks = (n + 1 + kg - 1) / kg;
    int32_t* off = plan + 8;
    int32_t* ksm = off + grid;
    int32_t* tg = ksm + grid;
    int32_t* tk = tg + grid;
    __shared__ int sTg, sNg;
    __shared__ int64_t carry;
    __shared__ int scan[WG];
    constexpr int MAXK = 1024;
    __shared__ int ck[MAXK];   // tiles read by each chunk
    for (int ks = tid; ks < nks && ks < MAXK; ks += WG) ck[ks] = cnt[min(ks * kg + kg - 1, n)];
    __syncthreads();
    if (tid < 64) {
        // One wavefront: workgroups used for Tg tiles per group are the sum over chunks of
        // ceil(cnt_ks / Tg); take the smallest Tg (binary search; the count does not grow with Tg) that
        // keeps them within G, so that the sweep runs in one round of the device.
        auto chunk = [&](int ks) -> int64_t { return ks < MAXK ? ck[ks] : cnt[min(ks * kg + kg - 1, n)]; };
        auto wsum = [&](int64_t v) {
            for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
            return v;
        };
        auto used = [&](int64_t t) {
            int64_t u = 0;
            for (int ks = tid; ks < nks; ks += 64) u += (chunk(ks) + t - 1) / t;
            return wsum(u);
        };
        int64_t W = 0;
        for (int ks = tid; ks < nks; ks += 64) W += chunk(ks);
        W = wsum(W);
        const int64_t cn = cnt[n];
        int64_t lo = W > G ? (W + G - 1) / G : 1, hi = cn > lo ? cn : lo;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (used(mid) <= G) hi = mid;
            else lo = mid + 1;
        }
        if (tid == 0) {
            sTg = (int)lo;
            sNg = (int)((cn + lo - 1) / lo);
            carry = 0;
        }
    }
    for (int64_t w = tid; w < grid; w += WG) tg[w] = -1;
    __syncthreads();
    const int Tg = sTg, ng = sNg;
    for (int base = 0; base < ng; base += WG) {
        const int g = base + tid;
        int nch = 0, km = 0;
        if (g < ng) {
            km = Dl[(int64_t)g * Tg] / kg;
            nch = nks - km;
        }
        scan[tid] = nch;
        __syncthreads();
        for (int d = 1; d < WG; d <<= 1) {
            const int v = tid >= d ? scan[tid - d] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const int64_t o = carry + scan[tid] - nch;
        if (g < ng) {
            off[g] = (int32_t)o;
            ksm[g] = km;
            for (int i = 0; i < nch; ++i)
                if (o + i < grid) {
                    tg[o + i] = g;
                    tk[o + i] = km + i;
                }
        }
        __syncthreads();
        if (tid == WG - 1) carry += scan[WG - 1];
        __syncthreads();
    }
    if (tid == 0) {
        plan[0] = ng;
        plan[1] = Tg;
        plan[2] = (int32_t)carry;
        plan[3] = nks;
    }
}

// Zero every row tile (4 * WG vectors of 16 bytes) whose nearest block row is
// within lim hops, in nsl slabs and in y; one workgroup per tile.
__global__ __launch_bounds__(WG) void k_zero_tiles(int64_t nbrow, int bpt, const int32_t* __restrict__ dist, int lim,
                                                   double2* __restrict__ base, int64_t slab_v, int nsl,
                                                   double2* __restrict__ y, int64_t nvec) {
    const int64_t t = blockIdx.x;
    const int64_t I0 = t * bpt, I1 = I0 + bpt < nbrow ? I0 + bpt : nbrow;
    int m = SUP_FAR;
    for (int64_t I = I0; I < I1; ++I) m = min(m, dist[I]);
    if (m > lim) return;
    const double2 z = make_double2(0.0, 0.0);
    for (int q = 0; q < 4; ++q) {
        const int64_t vi = t * (4 * WG) + q * WG + threadIdx.x;
        if (vi >= nvec) continue;
        for (int sl = 0; sl < nsl; ++sl) base[sl * slab_v + vi] = z;
        y[vi] = z;
    }
}

LaunchInfo launch_zero_ring(int64_t nbrow, const int32_t* brp, const int32_t* bcol, int32_t* dist, int hmax,
                            int bpt, void* base, int64_t slab_bytes, int nsl, void* y, int64_t nvec, hipStream_t s) {
    const unsigned rw = (unsigned)((nbrow + WG - 1) / WG);
    const int64_t ntiles = (nbrow + bpt - 1) / bpt;
    hipLaunchKernelGGL(k_sup_hop, dim3(rw), dim3(WG), 0, s, nbrow, brp, bcol, dist, hmax + 1);
    hipLaunchKernelGGL(k_zero_tiles, dim3((unsigned)ntiles), dim3(WG), 0, s, nbrow, bpt, dist, hmax + 1,
                       (double2*)base, slab_bytes / 16, nsl, (double2*)y, nvec);
    LaunchInfo li;
    li.wgs = ntiles;
    li.bytes = (double)nbrow * 8.0;
    return li;
}

// Local regions (order-N form): bit b of mask[I * W + b / 32] is set when block
// row I lies within r hops of the block of seed b. k_loc_seed marks the seeds'
// own blocks; each k_loc_hop adds the blocks one hop further (from a separate
// input buffer, so a launch moves exactly one hop).
__global__ __launch_bounds__(WG) void k_loc_seed(int64_t nbrow, int W, const int32_t* __restrict__ seeds, int ns,
                                                 int64_t M, uint32_t* __restrict__ mask) {
    const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (g >= nbrow * W) return;
    const int64_t I = g / W;
    const int w = (int)(g % W);
    uint32_t bits = 0;
    for (int i = 0; i < 32; ++i) {
        const int b = w * 32 + i;
        if (b < ns) {
            const int j = seeds[b];
            if (j >= 0 && j < M && j / 4 == I) bits |= 1u << i;
        }
    }
    mask[g] = bits;
}

__global__ __launch_bounds__(WG) void k_loc_hop(int64_t nbrow, int W, const int32_t* __restrict__ brp,
                                                const int32_t* __restrict__ bcol, const uint32_t* __restrict__ in,
                                                uint32_t* __restrict__ out) {
    const int64_t g = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (g >= nbrow * W) return;
    const int64_t I = g / W;
    const int w = (int)(g % W);
    uint32_t bits = in[g];
    const int lo = brp[I], hi = brp[I + 1];
    for (int p = lo; p < hi; ++p) bits |= in[(int64_t)bcol[p] * W + w];
    out[g] = bits;
}

const uint32_t* launch_local_masks(int64_t M, int64_t nbrow, const int32_t* brp, const int32_t* bcol,
                                   const int32_t* seeds, int ns, int W, int r, uint32_t* m0, uint32_t* m1,
                                   hipStream_t s) {
    const unsigned g = (unsigned)((nbrow * W + WG - 1) / WG);
    hipLaunchKernelGGL(k_loc_seed, dim3(g), dim3(WG), 0, s, nbrow, W, seeds, ns, M, m0);
    uint32_t* a = m0;
    uint32_t* b = m1;
    for (int h = 0; h < r; ++h) {
        hipLaunchKernelGGL(k_loc_hop, dim3(g), dim3(WG), 0, s, nbrow, W, brp, bcol, a, b);
        uint32_t* t = a;
        a = b;
        b = t;
    }
    return a;
}

LaunchInfo launch_projr_plan(const int32_t* cnt, const int32_t* Dl, int n0, int nsteps, int kg, int64_t G,
                             int64_t pstride, int32_t* plans, hipStream_t s) {
    LaunchInfo li;
    if (nsteps <= 0 || pstride < 8 + 4 * projr_sp_grid(G, n0 + nsteps, kg)) {
        li.wgs = nsteps <= 0 ? 0 : -1;
        return li;
    }
    hipLaunchKernelGGL(k_projr_plan, dim3((unsigned)nsteps), dim3(WG), 0, s, cnt, Dl, n0, kg, G, pstride, plans);
    li.wgs = nsteps;
    li.bytes = (double)nsteps * (double)pstride * 4.0;
    return li;
}

// red[(r * nk + k) * B + b] = sum over the groups that read slab k of the
// partial of workgroup off[g] + ks - ksmin[g] (ks = k / kg), in group order
// (group lanes strided by CL, then the CL lane sums in order).
template <int OPW>
__global__ __launch_bounds__(WG) void k_reduce_sp(const double* __restrict__ part, const int32_t* __restrict__ plan,
                                                  int64_t grid, int kg, int nk, int B, int64_t L,
                                                  double* __restrict__ out) {
    constexpr int CL = WG / OPW;
    const int oi = threadIdx.x % OPW, cl = threadIdx.x / OPW;
    const int64_t o = (int64_t)blockIdx.x * OPW + oi;
    const int ng = plan[0];
    const int32_t* off = plan + 8;
    const int32_t* ksm = off + grid;
    double s0 = 0.0;
    if (o < L) {
        const int64_t b = o % B, k = (o / B) % nk, r = o / ((int64_t)nk * B);
        const int ks = (int)(k / kg), kk = (int)(k % kg);
        for (int g = cl; g < ng; g += CL) {
            const int km = ksm[g];
            if (km <= ks) {
                const int64_t w = off[g] + (ks - km);
                s0 += part[((w * 3 + r) * kg + kk) * B + b];
            }
        }
    }
    __shared__ double lds[WG];
    lds[threadIdx.x] = s0;
    __syncthreads();
    if (cl == 0 && o < L) {
        double t = 0.0;
        for (int c = 0; c < CL; ++c) t += lds[c * OPW + oi];
        out[o] = t;
    }
}

LaunchInfo launch_reduce_sp(const double* part, const int32_t* plan, int64_t grid, int kg, int nk, int B,
                            double* out, hipStream_t s) {
    const int64_t L = (int64_t)3 * nk * B;
    LaunchInfo li;
    if (L <= 2048) {
        const int64_t wgs = (L + 3) / 4;
        hipLaunchKernelGGL((k_reduce_sp<4>), dim3(wgs), dim3(WG), 0, s, part, plan, grid, kg, nk, B, L, out);
        li.wgs = wgs;
    } else {
        const int64_t wgs = (L + 15) / 16;
        hipLaunchKernelGGL((k_reduce_sp<16>), dim3(wgs), dim3(WG), 0, s, part, plan, grid, kg, nk, B, L, out);
        li.wgs = wgs;
    }
    li.bytes = (double)L * 8.0;
    return li;
}

}  // namespace mar
