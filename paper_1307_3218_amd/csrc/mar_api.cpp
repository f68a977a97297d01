// Host side of the C ABI: argument validation, matrix upload (BSR 4x4 or CSR),
// the per-block launch sequence of the hot path, and per-kernel timing.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mar.h"
#include "mar_internal.h"

using mar::DevMat;
using mar::LaunchInfo;

namespace {

// One class per kernel variant, so that a class maps to one kernel symbol in a trace.
enum ProfClass {
    P_INIT = 0, P_SPMM, P_SPMM_DOT, P_PROJ2, P_PROJ1, P_UPD, P_REDUCE, P_NORM, P_APPEND, P_EIG, P_SUM,
    P_PROJR, P_UPD2, P_COEF, P_MU, P_SUPPORT, P_COUNT
};
const char* kProfNames[P_COUNT] = {"init",   "spmm",     "spmm_dot",  "cgs_proj_KSK", "cgs_proj_1",
                                   "cgs_upd", "reduce",  "norm",      "append",       "eig",
                                   "sum",     "dcgs_proj", "dcgs_upd", "dcgs_coef", "fermi_search",
                                   "support"};

// Launches restricted to a block's support record where the block's tile
// counts were copied (sp_cnt, device) and the step; the collector turns the
// full-sweep bytes and flops into the restricted ones.
enum SpKind { SP_NONE = 0, SP_PROJR, SP_UPD2, SP_UPD2_LAST, SP_FRAC };
struct ProfRec {
    int cls;
    hipEvent_t a, b;
    double bytes, flops;
    int sp = SP_NONE, sp_n = 0, sp_len = 0;
    const int32_t* sp_cnt = nullptr;
    double sp_unit = 0.0;     // bytes of one tile of one vector
    double sp_elem = 4.0;     // bytes of one element
    double sp_ntiles = 1.0;
};

thread_local std::string g_create_err;

std::string fmt(const char* f, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, f);
    vsnprintf(buf, sizeof buf, f, ap);
    va_end(ap);
    return buf;
}

}  // namespace

struct mar_ctx {
    int64_t M = 0;
    int device = 0;
    DevMat H, S;
    DevMat SH;                // S's values on H's BSR pattern (for the fused H/S product), if H is BSR
    int32_t* Hrp = nullptr;
    int32_t* Hcol = nullptr;
    double* Hval = nullptr;
    double* SvalH = nullptr;  // S on H's pattern (zeros where S stores nothing)
    double* diagS = nullptr;
    int64_t nnzH = 0, nnzS = 0;
    int max_row = 0;
    int n_cu = 1;             // compute units of the device
    bool dry = false;         // size and allocate the workspace only; launch nothing
    bool in_graph = false;    // sizing or capturing a mar_solve_many graph (one stream per system there)
    bool ran_two_sets = false;    // a solve ran two seed blocks in flight (mar_solve_many refuses the context)
    // projection workgroups per compute unit, by (element bytes, B, variant)
    std::map<std::tuple<int, int, int>, int> occ;
    // autotuned (B, projection variant) by (nu, precision)
    std::map<std::pair<int, int>, std::pair<int, int>> tuned;
    double* tune_buf = nullptr;   // probe outputs of the autotuner: rho [nnz(H)] + e_band
    double* zc_defer = nullptr;   // set during a solve whose assembly waits for a device Fermi level
    struct EsHook {               // eigen-state passes (mode 1: reference seed, 2: signed components)
        int mode = 0;
        double *Rg = nullptr, *Y = nullptr, *eps1 = nullptr, *yref = nullptr, *vref = nullptr;
        const double* lv = nullptr;
        double sigma = 0.0;
        double *pdot = nullptr, *pred = nullptr, *phi = nullptr;
        int groups = 64;
    } es;
    char* fws = nullptr;          // workspace of the device Fermi-level search
    size_t fws_bytes = 0;
    // local flipping: distance-2 colouring of H's rows (built at the first call) and workspace
    int32_t* fl_coff = nullptr;   // [ncol + 1]
    int32_t* fl_crow = nullptr;   // [M] rows by colour, index order within a colour
    int fl_ncol = 0;
    char* flws = nullptr;         // r, s [M] doubles and flags [M]

    mar_tuning tune{};
    int32_t loc = -1;             // local-region hops of later solves (< 0: the full system)
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* ext_ws = nullptr;       // a caller's workspace for the current solve (nothing is allocated then)
    size_t ext_bytes = 0;
    bool ext_short = false;       // the current solve needs more than ext_bytes
    char* ws_act = nullptr;       // the workspace the current solve runs on (ws or ext_ws)
    char* io = nullptr;
    size_t io_bytes = 0;
    hipStream_t stream = nullptr;
    hipStream_t stream2 = nullptr;   // second stream of the batched form (non-blocking): the eigensolves, or
                                     // every other seed block
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_eig[2] = {nullptr, nullptr};   // per eigensolve buffer
    std::string err;
    bool prof = false;
    bool refused = false;   // a launcher refused to run in the current solve
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> evfree;
    std::vector<void*> plogs;     // tile-count logs of profiled support-restricted solves
    mar_prof_entry agg[MAR_PROF_CLASSES];
    std::vector<void*> allocs;

    ~mar_ctx() {
        for (auto& r : recs) {
            hipEventDestroy(r.a);
            hipEventDestroy(r.b);
        }
        for (auto e : evfree) hipEventDestroy(e);
        for (void* p : plogs) hipFree(p);
        for (void* p : allocs) hipFree(p);
        if (ws) hipFree(ws);
        if (io) hipFree(io);
        if (fws) hipFree(fws);
        if (flws) hipFree(flws);
        if (stream) hipStreamDestroy(stream);
        if (stream2) hipStreamDestroy(stream2);
        if (ev_fork) hipEventDestroy(ev_fork);
        if (ev_join) hipEventDestroy(ev_join);
        for (int i = 0; i < 2; ++i) {
            if (ev_ready[i]) hipEventDestroy(ev_ready[i]);
            if (ev_eig[i]) hipEventDestroy(ev_eig[i]);
        }
    }
};

namespace {

mar_status set_err(mar_ctx* c, mar_status st, const std::string& m) {
    if (c) c->err = m;
    else g_create_err = m;
    return st;
}

#define HIP_OR(c, call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return set_err(c, e_ == hipErrorOutOfMemory ? MAR_ERR_NOMEM : MAR_ERR_HIP,               \
                           fmt("%s failed: %s", #call, hipGetErrorString(e_)));                      \
    } while (0)

// ---------------------------------------------------------------- validation
mar_status check_csr(int64_t M, const int64_t* rp, const int32_t* col, const double* val, const char* nm,
                     std::string& msg) {
    if (!rp) return msg = fmt("%s: rowptr is NULL", nm), MAR_ERR_ARG;
    if (rp[0] != 0) return msg = fmt("%s: rowptr[0] = %lld, expected 0", nm, (long long)rp[0]), MAR_ERR_PATTERN;
    for (int64_t i = 0; i < M; ++i)
        if (rp[i + 1] < rp[i]) return msg = fmt("%s: rowptr decreases at row %lld", nm, (long long)i), MAR_ERR_PATTERN;
    const int64_t nnz = rp[M];
    if (nnz >= (int64_t)INT32_MAX) return msg = fmt("%s: nnz %lld exceeds int32 range", nm, (long long)nnz), MAR_ERR_ARG;
    if (nnz > 0 && (!col || !val)) return msg = fmt("%s: col or val is NULL", nm), MAR_ERR_ARG;
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
            if (col[t] < 0 || col[t] >= M)
                return msg = fmt("%s: column %d out of range in row %lld", nm, col[t], (long long)i), MAR_ERR_PATTERN;
            if (t > rp[i] && col[t] <= col[t - 1])
                return msg = fmt("%s: columns not sorted/unique in row %lld", nm, (long long)i), MAR_ERR_PATTERN;
            if (!std::isfinite(val[t]))
                return msg = fmt("%s: non-finite value at (%lld, %d)", nm, (long long)i, col[t]), MAR_ERR_ARG;
        }
    }
    return MAR_OK;
}

int64_t find_slot(const int64_t* rp, const int32_t* col, int64_t i, int32_t j) {
    const int32_t* lo = col + rp[i];
    const int32_t* hi = col + rp[i + 1];
    const int32_t* p = std::lower_bound(lo, hi, j);
    return (p != hi && *p == j) ? (p - col) : -1;
}

mar_status check_sym(int64_t M, const int64_t* rp, const int32_t* col, const double* val, const char* nm,
                     std::string& msg) {
    for (int64_t i = 0; i < M; ++i)
        for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
            const int64_t u = find_slot(rp, col, col[t], (int32_t)i);
            if (u < 0)
                return msg = fmt("%s: pattern not symmetric at (%lld, %d)", nm, (long long)i, col[t]), MAR_ERR_PATTERN;
            if (val[u] != val[t])
                return msg = fmt("%s: values not symmetric at (%lld, %d)", nm, (long long)i, col[t]), MAR_ERR_PATTERN;
        }
    return MAR_OK;
}

// 4x4 block structure: rows 4I..4I+3 share one pattern made of aligned groups of 4.
bool detect_bsr4(int64_t M, const int64_t* rp, const int32_t* col) {
    if (M % 4 != 0) return false;
    for (int64_t I = 0; I < M / 4; ++I) {
        const int64_t L = rp[4 * I + 1] - rp[4 * I];
        if (L % 4 != 0) return false;
        for (int r = 1; r < 4; ++r) {
            if (rp[4 * I + r + 1] - rp[4 * I + r] != L) return false;
            if (std::memcmp(col + rp[4 * I], col + rp[4 * I + r], L * sizeof(int32_t)) != 0) return false;
        }
        for (int64_t t = 0; t < L; t += 4) {
            const int32_t c0 = col[rp[4 * I] + t];
            if (c0 % 4 != 0) return false;
            for (int q = 1; q < 4; ++q)
                if (col[rp[4 * I] + t + q] != c0 + q) return false;
        }
    }
    return true;
}

template <typename X>
mar_status upload(mar_ctx* c, X** dst, const X* src, size_t n) {
    *dst = nullptr;
    if (n == 0) n = 1;
    void* p = nullptr;
    HIP_OR(c, hipMalloc(&p, n * sizeof(X)));
    c->allocs.push_back(p);
    *dst = (X*)p;
    if (src) HIP_OR(c, hipMemcpy(p, src, n * sizeof(X), hipMemcpyHostToDevice));
    return MAR_OK;
}

mar_status build_devmat(mar_ctx* c, int64_t M, const int64_t* rp, const int32_t* col, const double* val, DevMat& D) {
    mar_status st;
    if (detect_bsr4(M, rp, col)) {
        const int64_t nb = M / 4, nblk = rp[M] / 16;
        std::vector<int32_t> brp(nb + 1), bcol(nblk);
        std::vector<double> v64(nblk * 16);
        std::vector<float> v32(nblk * 16);
        for (int64_t I = 0; I <= nb; ++I) brp[I] = (int32_t)(rp[4 * std::min(I, nb)] / 16);
        for (int64_t I = 0; I < nb; ++I) {
            const int64_t L = rp[4 * I + 1] - rp[4 * I];
            for (int64_t t = 0; t < L / 4; ++t) {
                const int64_t blk = brp[I] + t;
                bcol[blk] = col[rp[4 * I] + 4 * t] / 4;
                for (int r = 0; r < 4; ++r)
                    for (int q = 0; q < 4; ++q) {
                        const double x = val[rp[4 * I + r] + 4 * t + q];
                        v64[blk * 16 + r * 4 + q] = x;
                        v32[blk * 16 + r * 4 + q] = (float)x;
                    }
            }
        }
        D.bsr = true;
        D.n = nb;
        D.nnz = nblk;
        std::vector<int64_t> off;
        off.reserve((size_t)nblk);
        for (int64_t I = 0; I < nb; ++I)
            for (int64_t b = brp[I]; b < brp[I + 1]; ++b)
                if (bcol[b] != I) off.push_back(std::llabs((int64_t)bcol[b] - I));
        if (!off.empty()) {
            auto q = off.begin() + (ptrdiff_t)(off.size() * 9 / 10);
            std::nth_element(off.begin(), q, off.end());
            D.span = *q;
        }
        if ((st = upload(c, &D.ptr, brp.data(), brp.size())) != MAR_OK) return st;
        if ((st = upload(c, &D.idx, bcol.data(), bcol.size())) != MAR_OK) return st;
        if ((st = upload(c, &D.v64, v64.data(), v64.size())) != MAR_OK) return st;
        if ((st = upload(c, &D.v32, v32.data(), v32.size())) != MAR_OK) return st;
    } else {
        const int64_t nnz = rp[M];
        std::vector<int32_t> rp32(M + 1);
        for (int64_t i = 0; i <= M; ++i) rp32[i] = (int32_t)rp[i];
        std::vector<float> v32(nnz);
        for (int64_t t = 0; t < nnz; ++t) v32[t] = (float)val[t];
        D.bsr = false;
        D.n = M;
        D.nnz = nnz;
        if ((st = upload(c, &D.ptr, rp32.data(), rp32.size())) != MAR_OK) return st;
        if ((st = upload(c, &D.idx, col, (size_t)nnz)) != MAR_OK) return st;
        if ((st = upload(c, &D.v64, val, (size_t)nnz)) != MAR_OK) return st;
        if ((st = upload(c, &D.v32, v32.data(), v32.size())) != MAR_OK) return st;
    }
    return MAR_OK;
}

// ---------------------------------------------------------------- profiling
hipEvent_t get_event(mar_ctx* c) {
    if (!c->evfree.empty()) {
        hipEvent_t e = c->evfree.back();
        c->evfree.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

// Runs one launcher; a launcher that refuses (partial-sum buffer too small)
// marks the solve as failed, and no later kernel of the solve is enqueued.
// Bytes and flops of a support-restricted launch from its block's tile counts
// cnt[h] (tiles with distance <= h): every slab and right-hand side read once
// on the tiles where it can be nonzero, every result written once there.
void support_figures(ProfRec& r, const std::vector<int32_t>& cnt) {
    const int n = r.sp_n, hmax = (int)cnt.size() - 1;
    auto at = [&](int h) { return (double)cnt[(size_t)std::min(std::max(h, 0), hmax)]; };
    double below = 0.0;   // sum of cnt[k] over k < n
    for (int k = 0; k < n; ++k) below += at(k);
    const double el = r.sp_unit / r.sp_elem;   // elements of one tile of one vector
    switch (r.sp) {
        case SP_PROJR:       // slabs 0..n and three right-hand sides
            r.bytes = (below + at(n) + 3.0 * at(n)) * r.sp_unit;
            r.flops = 6.0 * (below + at(n)) * el;
            break;
        case SP_UPD2:        // slabs 0..n-1, u~ and y read; u_n and w' written
            r.bytes = (below + 2.0 * at(n) + 2.0 * at(n + 1)) * r.sp_unit;
            r.flops = 4.0 * below * el;
            break;
        case SP_UPD2_LAST:   // slabs 0..n-1 and u~ read; u_n written
            r.bytes = (below + 2.0 * at(n)) * r.sp_unit;
            r.flops = 2.0 * below * el;
            break;
        case SP_FRAC: {      // rows of the tiles within distance n
            const double f = at(n) / r.sp_ntiles;
            r.bytes *= f;
            r.flops *= f;
            break;
        }
        default: break;
    }
}

// Returns whether a profile record was added (the last one of c->recs).
template <class F>
bool launch(mar_ctx* c, hipStream_t s, int cls, F&& f) {
    if (c->refused || c->dry) return false;
    if (!c->prof) {
        if (f().wgs < 0) c->refused = true;
        return false;
    }
    hipEvent_t a = get_event(c), b = get_event(c);
    hipEventRecord(a, s);
    LaunchInfo li = f();
    hipEventRecord(b, s);
    if (li.wgs < 0) c->refused = true;
    ProfRec r;
    r.cls = cls;
    r.a = a;
    r.b = b;
    r.bytes = li.bytes;
    r.flops = li.flops;
    c->recs.push_back(r);
    return true;
}

// ---------------------------------------------------------------- block size
int pow2_floor(int64_t x) {
    int p = 1;
    while ((int64_t)p * 2 <= x) p *= 2;
    return p;
}

// Widest block whose stored basis (K, plus S K in the textbook schedule) fits in 128 GB.
int block_cap(const mar_ctx* c, int nu, mar_precision prec, bool delayed) {
    const int bmax = prec == MAR_FP32 ? mar::max_block<float>() : mar::max_block<double>();
    const double p = prec == MAR_FP32 ? 4.0 : 8.0, copies = delayed ? 1.0 : 2.0;
    int B = bmax;
    while (B > 1 && copies * nu * (double)c->M * B * p > 128e9) B /= 2;
    return B;
}

int choose_block(const mar_ctx* c, int nu, mar_precision prec, int64_t n_seeds, bool delayed) {
    const int bmax = prec == MAR_FP32 ? mar::max_block<float>() : mar::max_block<double>();
    int B;
    if (c->tune.seed_block > 0) {
        B = std::min(c->tune.seed_block, bmax);
    } else {
        auto t = c->tuned.find({nu, (int)prec});
        if (t != c->tuned.end() && delayed) {
            B = t->second.first;
        } else {
            // the widest block: one pass over a slab serves the most seeds and
            // the matrix values are reused B times
            B = block_cap(c, nu, prec, delayed);
        }
        if (n_seeds > 0) B = std::min<int64_t>(B, pow2_floor(std::max<int64_t>(1, n_seeds)) * 2);
        B = std::min(B, bmax);
    }
    return std::max(1, pow2_floor(B));
}

// What a solve will run: block size, schedule and projection variant.
struct Plan {
    int B;
    bool delayed;
    int variant;
};

Plan plan_solve(const mar_ctx* c, int nu, mar_precision prec, mar_form form, int64_t n_seeds) {
    Plan pl;
    // the plain form is the textbook CGS2 (project, update, project, update);
    // the batched form defaults to the delayed-reorthogonalization schedule
    pl.delayed = c->tune.schedule == MAR_SCHED_DELAYED ||
                 (c->tune.schedule == MAR_SCHED_AUTO && form == MAR_FORM_BATCHED);
    pl.B = form == MAR_FORM_PLAIN ? 1 : choose_block(c, nu, prec, n_seeds, pl.delayed);
    pl.variant = c->tune.proj_variant;
    if (pl.variant == 0 && c->tune.seed_block == 0 && form == MAR_FORM_BATCHED) {
        auto t = c->tuned.find({nu, (int)prec});
        if (t != c->tuned.end()) pl.variant = t->second.second;
    }
    return pl;
}

// Projection workgroups one compute unit holds (cached per kernel instance).
template <typename T>
int projr_occupancy(mar_ctx* c, int B, int variant) {
    const auto key = std::make_tuple((int)sizeof(T), B, variant);
    auto it = c->occ.find(key);
    if (it != c->occ.end()) return it->second;
    const int nb = mar::projr_blocks_per_cu<T>(B, variant);
    c->occ[key] = nb;
    return nb;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Elements between consecutive basis slabs: M*B plus a pad (1 KiB unless tuned), so that the same row of
// different slabs does not sit at a power-of-two distance (at M*B*4 = 2^27 bytes the projection, which reads
// four slabs at one row offset, ran 3 % slower without it).
int64_t slab_stride(const mar_ctx* c, int64_t Mp, int B, size_t elem) {
    const int64_t pad_bytes = (int64_t)(c->tune.slab_pad_kb > 0 ? c->tune.slab_pad_kb : 1) * 1024;
    return Mp * B + pad_bytes / (int64_t)elem;
}

void drop_graphs_of(mar_ctx* c);

mar_status ensure_ws(mar_ctx* c, size_t bytes) {
    if (c->ext_ws) {   // the caller's workspace: never allocate, refuse what does not fit
        c->ws_act = c->ext_ws;
        if (bytes <= c->ext_bytes) return MAR_OK;
        c->ext_short = true;
        return set_err(c, MAR_ERR_ARG,
                       fmt("the solve needs %zu bytes of workspace, more than the %zu bytes of the static scratch",
                           bytes, c->ext_bytes));
    }
    c->ws_act = c->ws;
    if (bytes <= c->ws_bytes) return MAR_OK;
    if (c->ws) {
        HIP_OR(c, hipDeviceSynchronize());
        drop_graphs_of(c);   // cached graphs hold pointers into the old workspace
        HIP_OR(c, hipFree(c->ws));
        c->ws = nullptr;
        c->ws_bytes = 0;
    }
    void* p = nullptr;
    HIP_OR(c, hipMalloc(&p, bytes));
    c->ws = (char*)p;
    c->ws_bytes = bytes;
    c->ws_act = c->ws;
    return MAR_OK;
}

// ---------------------------------------------------------------- the solve
// The eigensolve and assembly of one seed block, or one of the eigen-state passes.
template <typename T>
void eig_stage(mar_ctx* c, hipStream_t s, int B, int ns, const int32_t* seeds, int nu, double* h, const int32_t* nucp,
               const double* Kp, const T* K, int64_t stride, int64_t Mp, double mu, double kT, double* rho,
               double* e_seed, double* n_seed, int32_t* nu_out, double* eps, double* w, int64_t blk0) {
    mar::EigExtra ex;
    ex.eig_max_sweeps = c->tune.eig_max_sweeps > 0 ? c->tune.eig_max_sweeps : 40;
    if (c->es.mode == 2) {   // v_ref . v_alpha^(j) through K^T v_ref, then the signed Eq. 3 component
        launch(c, s, P_EIG, [&] {
            return mar::launch_es_pdot<T>(B, K, stride, c->M, Mp, nu, c->es.vref, c->es.pdot, c->es.groups, s);
        });
        launch(c, s, P_REDUCE, [&] {
            return mar::launch_reduce(c->es.pdot, c->es.groups, (int64_t)nu * B, c->es.pred, nullptr, B, nu, 0, s);
        });
        ex.mode = 2;
        ex.pref = c->es.pred;
        ex.pB = B;
        ex.win = c->es.lv;
        ex.sigma = c->es.sigma;
        ex.phi = c->es.phi + blk0;
    } else if (c->es.mode == 1) {   // the reference seed's full subspace eigenvectors
        ex.mode = 1;
        ex.Rg = c->es.Rg;
        ex.Y = c->es.Y;
        eps = c->es.eps1;
        w = nullptr;
    }
    launch(c, s, P_EIG, [&] {
        return mar::launch_eig(ns, seeds, nu, h, nucp, Kp, c->Hrp, c->Hcol, c->Hval, c->SvalH, c->diagS, c->max_row,
                               mu, kT, rho, e_seed, n_seed, nu_out, eps, w,
                               c->zc_defer ? c->zc_defer + (size_t)blk0 * nu * c->max_row : nullptr, ex, s);
    });
    if (c->es.mode == 1)
        launch(c, s, P_EIG, [&] {
            return mar::launch_es_refvec<T>(K, stride, c->M, seeds, nu, nucp, c->es.Y, c->es.eps1, c->es.lv,
                                            c->es.sigma, c->es.yref, c->es.vref, s);
        });
}

template <typename T>
mar_status run_solve(mar_ctx* c, const int32_t* d_seeds, int64_t n_seeds, int nu, double mu, double kT, int B,
                     double* d_rho, double* d_e_band, double* d_e_seed, double* d_n_seed, int32_t* d_nu_eff,
                     double* d_eps, double* d_w, hipStream_t s) {
    constexpr int VEC = 16 / sizeof(T);
    // vectors are stored with the row count padded to a multiple of 4, so that
    // every [M][B] array is a whole number of 16-byte vectors; padded rows stay 0
    const int64_t M = (c->M + 3) / 4 * 4;
    const int64_t nvec = M * B / VEC;
    const int64_t chunks = (nvec + mar::WG * mar::PROJ_Q - 1) / (mar::WG * mar::PROJ_Q);
    const int P = B < VEC ? 1 : B / VEC;
    const int64_t spmm_wgs = std::max((c->S.n * P + mar::WG - 1) / mar::WG, (c->H.n * P + mar::WG - 1) / mar::WG);
    const size_t slab = (size_t)M * B * sizeof(T);
    const int64_t stride = slab_stride(c, M, B, sizeof(T));

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t oK = take((size_t)nu * stride * sizeof(T)), oSK = take((size_t)nu * stride * sizeof(T));
    const size_t oW = take(slab), oZ = take(slab);
    const int64_t part_cap = (int64_t)std::max<size_t>((size_t)chunks * 2 * nu * B, (size_t)spmm_wgs * B);
    const size_t oPart = take((size_t)part_cap * 8);
    const size_t oRed1 = take((size_t)2 * nu * B * 8), oRed2 = take((size_t)nu * B * 8), oRedb = take((size_t)B * 8);
    const size_t oH = take((size_t)B * nu * nu * 8), oBeta = take((size_t)B * 8);
    const size_t oAct = take((size_t)B * 4), oNu = take((size_t)B * 4);
    const size_t oKp = take((size_t)B * nu * std::max(1, c->max_row) * 8), oNuCp = take((size_t)B * 4);
    const bool own_e = d_e_seed == nullptr, own_n = d_n_seed == nullptr, own_nu = d_nu_eff == nullptr;
    const size_t oE = take(own_e ? (size_t)n_seeds * 8 : 0), oN = take(own_n ? (size_t)n_seeds * 8 : 0);
    const size_t oNuOut = take(own_nu ? (size_t)n_seeds * 4 : 0);
    // With two or more blocks each block's eigensolve runs on the second stream while the next block's
    // steps run on the caller's (as in the delayed schedule): the subspace matrix and the gathered rows
    // alternate between two copies. Not while profiling, inside graphs, when the caller's stream is
    // capturing, for the eigen-state passes, or with tuning two_streams 1 or 2.
    const int64_t n_blocks = (n_seeds + B - 1) / B;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = !c->dry && hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
    const bool eig_ovl = n_blocks >= 2 && !c->prof && !c->in_graph && !capturing && c->es.mode == 0 &&
                         (c->tune.two_streams == 0 || c->tune.two_streams == 3) && c->stream2;
    const size_t oH2 = take(eig_ovl ? (size_t)B * nu * nu * 8 : 0);
    const size_t oKp2 = take(eig_ovl ? (size_t)B * nu * std::max(1, c->max_row) * 8 : 0);
    const size_t oNc2 = take(eig_ovl ? (size_t)B * 4 : 0);
    mar_status st = ensure_ws(c, off);
    if (st != MAR_OK) return st;
    char* w = c->ws_act;
    mar::BlockWS<T> ws{(T*)(w + oK), (T*)(w + oSK), (T*)(w + oW), (T*)(w + oZ), (double*)(w + oPart),
                       (double*)(w + oRed1), (double*)(w + oRed2), (double*)(w + oRedb), (double*)(w + oH),
                       (double*)(w + oBeta), (int32_t*)(w + oAct), (int32_t*)(w + oNu)};
    double* e_seed = own_e ? (double*)(w + oE) : d_e_seed;
    double* n_seed = own_n ? (double*)(w + oN) : d_n_seed;
    int32_t* nu_out = own_nu ? (int32_t*)(w + oNuOut) : d_nu_eff;
    const double tau = sizeof(T) == 4 ? 1e-5 : 1e-12;
    const int64_t slab_el = stride;

    for (int64_t blk0 = 0; blk0 < n_seeds; blk0 += B) {
        const int ns = (int)std::min<int64_t>(B, n_seeds - blk0);
        const int32_t* seeds = d_seeds + blk0;
        // overlapped eigensolves: odd blocks use the second copy of h and the gathered rows, and a block waits
        // until the eigensolve of the block before last has released its copy
        const int64_t bi = blk0 / B;
        const int ep = (int)(bi % 2);
        double* h = eig_ovl && ep == 1 ? (double*)(w + oH2) : ws.h;
        double* Kp = eig_ovl && ep == 1 ? (double*)(w + oKp2) : (double*)(w + oKp);
        int32_t* nucp = eig_ovl && ep == 1 ? (int32_t*)(w + oNc2) : (int32_t*)(w + oNuCp);
        if (eig_ovl && bi >= 2 && !c->dry) hipStreamWaitEvent(s, c->ev_eig[ep], 0);
        if (M != c->M && blk0 == 0) {
            // padded rows of W, Z and S K_1 must read as zero (spmm writes rows < M only)
            launch(c, s, P_INIT, [&] { return mar::launch_zero(ws.W, (int64_t)slab, s); });
            launch(c, s, P_INIT, [&] { return mar::launch_zero(ws.Z, (int64_t)slab, s); });
            launch(c, s, P_INIT, [&] { return mar::launch_zero(ws.SK, (int64_t)slab, s); });
        }
        launch(c, s, P_INIT, [&] {
            return mar::launch_init<T>(B, M, c->M, seeds, ns, c->diagS, nu, ws.K, ws.active, ws.nu_eff, nullptr, s);
        });
        launch(c, s, P_SPMM, [&] { return mar::launch_spmm<T>(B, c->S, ws.K, ws.SK, nullptr, 0, 0, s); });
        for (int n = 0; n < nu; ++n) {
            const T* Kn = ws.K + (size_t)n * slab_el;
            const int nk = n + 1;
            const bool last = n + 1 == nu;
            launch(c, s, P_SPMM, [&] { return mar::launch_spmm<T>(B, c->H, Kn, ws.W, nullptr, 0, 0, s); });
            // h[:, n] = K^T w and c1 = (S K)^T w in one pass over K and S K
            int64_t nch = 0;
            launch(c, s, last ? P_PROJ1 : P_PROJ2, [&] {
                return mar::launch_proj<T>(B, last ? 1 : 2, ws.K, ws.SK, M, stride, nk, ws.W, ws.part, part_cap,
                                           &nch, s);
            });
            const int64_t L1 = (int64_t)(last ? 1 : 2) * nk * B;
            launch(c, s, P_REDUCE, [&] { return mar::launch_reduce(ws.part, nch, L1, ws.red1, h, B, nu, n, s); });
            if (last) break;
            const double* c1 = ws.red1 + (size_t)nk * B;
            // CGS pass 1: w -= K c1
            launch(c, s, P_UPD, [&] { return mar::launch_upd<T>(B, ws.K, M, stride, nk, c1, ws.W, s); });
            // CGS pass 2: c2 = (S K)^T w, w -= K c2
            launch(c, s, P_PROJ1, [&] {
                return mar::launch_proj<T>(B, 1, ws.SK, nullptr, M, stride, nk, ws.W, ws.part, part_cap, &nch, s);
            });
            const int64_t L2 = (int64_t)nk * B;
            launch(c, s, P_REDUCE, [&] { return mar::launch_reduce(ws.part, nch, L2, ws.red2, nullptr, B, nu, n, s); });
            launch(c, s, P_UPD, [&] { return mar::launch_upd<T>(B, ws.K, M, stride, nk, ws.red2, ws.W, s); });
            // z = S w and w^T S w
            int64_t swgs = 0;
            launch(c, s, P_SPMM_DOT, [&] {
                LaunchInfo li = mar::launch_spmm<T>(B, c->S, ws.W, ws.Z, ws.part, 1, part_cap, s);
                swgs = li.wgs;
                return li;
            });
            launch(c, s, P_REDUCE, [&] { return mar::launch_reduce(ws.part, swgs, B, ws.redb, nullptr, B, nu, n, s); });
            launch(c, s, P_NORM, [&] {
                return mar::launch_norm(B, nk, ws.redb, c1, ws.red2, tau, ws.active, ws.nu_eff, ws.beta, n, s);
            });
            launch(c, s, P_APPEND, [&] {
                return mar::launch_append<T>(B, M, ws.W, ws.Z, ws.beta, ws.active, ws.K + (size_t)(n + 1) * slab_el,
                                             ws.SK + (size_t)(n + 1) * slab_el, s);
            });
        }
        launch(c, s, P_EIG, [&] {
            return mar::launch_gather<T>(B, ns, seeds, nu, ws.nu_eff, ws.K, stride, c->Hrp, c->Hcol, c->max_row, Kp,
                                         nucp, s);
        });
        hipStream_t se = s;
        if (eig_ovl && !c->dry) {   // the eigensolve reads only h, the gathered rows and H: off the caller's stream
            hipEventRecord(c->ev_ready[ep], s);
            hipStreamWaitEvent(c->stream2, c->ev_ready[ep], 0);
            se = c->stream2;
        }
        eig_stage<T>(c, se, B, ns, seeds, nu, h, nucp, Kp, ws.K, stride, M, mu, kT, d_rho, e_seed + blk0,
                     n_seed + blk0, nu_out + blk0, d_eps ? d_eps + blk0 * nu : nullptr,
                     d_w ? d_w + blk0 * nu : nullptr, blk0);
        if (eig_ovl && !c->dry) hipEventRecord(c->ev_eig[ep], c->stream2);
    }
    if (eig_ovl && !c->dry) {   // the caller's stream waits for the second stream's work
        hipEventRecord(c->ev_join, c->stream2);
        hipStreamWaitEvent(s, c->ev_join, 0);
    }
    if (!c->zc_defer && !c->es.mode) launch(c, s, P_SUM, [&] { return mar::launch_sum(e_seed, n_seeds, d_e_band, s); });
    if (c->refused) {
        c->refused = false;
        return set_err(c, MAR_ERR_STATE, "internal error: a partial-sum buffer was too small; solve not run");
    }
    HIP_OR(c, hipGetLastError());
    return MAR_OK;
}

// The delayed-reorthogonalization schedule (basis K only): per step two SpMMs
// on the once-orthogonalized vector (y = H u~, S y), one projection sweep over
// K with three right-hand sides, the FP64 coefficient kernel, one dual update
// sweep (second pass of u~ and first pass of y), then the S-norm of the new
// residual. Two passes over the basis per step instead of five.
template <typename T>
mar_status run_solve_delayed(mar_ctx* c, const int32_t* d_seeds, int64_t n_seeds, int nu, double mu, double kT,
                             int B, int variant, double* d_rho, double* d_e_band, double* d_e_seed,
                             double* d_n_seed, int32_t* d_nu_eff, double* d_eps, double* d_w, hipStream_t s) {
    constexpr int VEC = 16 / sizeof(T);
    const int64_t M = (c->M + 3) / 4 * 4;
    const int64_t nvec = M * B / VEC;
    const int P = B < VEC ? 1 : B / VEC;
    const int64_t spmm_wgs = std::max((c->S.n * P + mar::WG - 1) / mar::WG, (c->H.n * P + mar::WG - 1) / mar::WG);
    const size_t slab = (size_t)M * B * sizeof(T);
    const int64_t stride = slab_stride(c, M, B, sizeof(T));
    // H u and S u of the same vector in one pass when H is BSR (S on H's pattern)
    const bool dual = c->H.bsr && c->SH.nnz == c->H.nnz && B >= VEC;
    // Support tracking: the kernels of a step skip the row tiles on which the block's vectors are exactly
    // zero (farther from every seed of the block than the step in hops of H's pattern).
    const bool sparse = dual && c->tune.support_off == 0;
    const int64_t nbrow = c->H.n, bpt = mar::WG / std::max(P, 1);
    // local regions (order-N form): per block row and seed, inside the seed's region or not. With the support
    // tracking on, the products and the update then run over the support list (a small grid of kListWgs
    // workgroups in a grid-stride loop) instead of a workgroup per row tile of the whole cell.
    const bool local = c->loc >= 0 && dual;
    // Variant 0 streams the basis (variant 7: 8 slabs per workgroup, non-temporal loads) when the solve's
    // widest sweep (nu + 3 slabs) exceeds the last-level cache: each slab is read once per sweep, and
    // cached loads would only displace the lines that are reused (the right-hand sides, the vectors just
    // written). Decided once per solve, so that every projection of a solve runs one kernel on one plan.
    // Local regions sweep few tiles, which stay cached. Four slabs per workgroup (variant 2) instead:
    //  * at nu <= 64, where the sweeps are short: at nu = 30 on the 16384-row cell 8 slabs took the
    //    projection from 71 to 85 ms per step, where at nu = 100 on the 131072-row lattice they took it
    //    from 316 to 297 ms;
    //  * for the FP32 form at nu > kUpdAcc64Nu: there a single rho column's error depends on how the
    //    projection's FP32 sums are partitioned, and the 4-slab partition is the one measured within 1e-5
    //    (at nu = 300 on the 1048576-row lattice the worst of 8 sampled columns is 9.6e-6 with 4 slabs,
    //    2.9e-5 with 8).
    const bool four = nu <= 64 || (std::is_same<T, float>::value && nu > mar::kUpdAcc64Nu);
    const int pvar = variant == 0 && !local && (double)(nu + 3) * (double)slab > mar::kNtSweepBytes
                         ? (four ? 2 : 7)
                         : variant;
    const int kg = mar::projr_kg(pvar);
    // default projection grid: the workgroups the device holds at once (one round, few partial sums)
    const int64_t target = c->tune.proj_wgs > 0 ? (int64_t)c->tune.proj_wgs
                                                 : (int64_t)projr_occupancy<T>(c, B, pvar) * c->n_cu;
    // grid of the list kernels (local regions): each workgroup also leaves a row of S-norm partials, so small
    // regions run best on few workgroups (512: +2-7 % against 2048 at 4-10 hops, equal at 16, -2 % at 24)
    const int64_t kListWgs = c->loc >= 0 && c->loc <= 16 ? 512 : 2048;
    constexpr double kTwoSetBytes = 160e9;   // two seed-block workspaces only when both fit in this
    const int mW = (B + 31) / 32;
    const int hreach = local ? std::min(nu, (int)c->loc) : nu;   // farthest hop a vector can reach
    // Hops the support search covers. The whole-cell form does not clear the basis per block: the update
    // writes zeros into slab n + 1 on the tiles 1..kg hops past its support, the farthest a later sweep reads
    // it (a projection chunk of kg slabs, the fused product's neighbour rows), so the search runs kg + 1 hops
    // past the last vector. The eigen-state passes project whole slabs and clear the basis instead.
    const bool ring = sparse && !local && c->es.mode == 0;
    const int hsup = ring ? nu + kg + 1 : hreach;
    const int64_t ntiles = (nbrow + bpt - 1) / bpt;
    const int64_t grid_max = mar::projr_sp_grid(target, nu, kg);
    size_t part_doubles = 0;
    // S-norm partials of the fused product, one slot per workgroup (reduced into redb before the projection,
    // with part as the reduction's scratch)
    const size_t np_doubles = (size_t)std::max<int64_t>(spmm_wgs, kListWgs) * 2 * B;
    const int64_t np_cap = (int64_t)np_doubles;
    for (int nk = 1; nk <= nu; ++nk) {
        const mar::ProjrGeom gm = mar::projr_geometry(nvec, nk, pvar, target);
        part_doubles = std::max<size_t>(part_doubles, (size_t)gm.groups * 3 * nk * B);
    }
    if (sparse) part_doubles = std::max<size_t>(part_doubles, (size_t)grid_max * 3 * kg * B);
    // update depth of the full sweep (support tracking runs one tile of 4 * WG vectors per workgroup)
    const int upd_q = c->tune.upd_q > 0 ? c->tune.upd_q : 4;
    // the FP32 form's update sums in FP64 at large subspace dimensions
    const bool upd_acc64 = std::is_same<T, float>::value && nu > mar::kUpdAcc64Nu;
    const int64_t part_cap = (int64_t)part_doubles;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    // Per-set arrays (everything a seed block works on); with two sets, consecutive blocks alternate between
    // them and between the caller's stream and the context's second stream, so that one block's short FP64
    // kernels (reductions, coefficients, norms, eigensolver) overlap the other block's streaming sweeps.
    const size_t oK = take((size_t)nu * stride * sizeof(T)), oY = take(slab), oSY = take(slab), oZT = take(slab);
    const size_t oPart = take(part_doubles * 8), oNP = take(np_doubles * 8);
    const size_t oRed = take((size_t)3 * nu * B * 8), oRedb = take((size_t)2 * B * 8);
    const size_t oH = take((size_t)B * nu * nu * 8), oG = take((size_t)B * nu * nu * 8);
    const size_t oKp = take((size_t)B * nu * std::max(1, c->max_row) * 8), oNc = take((size_t)B * 4);
    const size_t oR = take((size_t)B * nu * (nu + 1) * 8), oC1 = take((size_t)B * nu * 8);
    const size_t oBT = take((size_t)B * 8), oUU = take((size_t)B * 8), oGam = take((size_t)B * 8),
                 oFn = take((size_t)B * 8);
    const size_t oCA = take((size_t)nu * B * 8), oCB = take((size_t)nu * B * 8);
    const size_t oCAf = take((size_t)nu * B * 4), oCBf = take((size_t)nu * B * 4);
    const size_t oAct = take((size_t)B * 4), oNu = take((size_t)B * 4);
    const size_t oDist = take(sparse ? (size_t)nbrow * 4 : 0), oTD = take(sparse ? (size_t)ntiles * 4 : 0);
    const size_t oCnt = take(sparse ? (size_t)(std::max(hsup, nu) + 1) * 4 : 0);
    const size_t oList = take(sparse ? (size_t)ntiles * 4 : 0);
    const int64_t pstride = 8 + 4 * grid_max;   // ints per projection plan; the plans of all steps are kept
    const size_t oDl = take(sparse ? (size_t)ntiles * 4 : 0), oPlan = take(sparse ? (size_t)nu * pstride * 4 : 0);
    const size_t oM0 = take(local ? (size_t)nbrow * mW * 4 : 0), oM1 = take(local ? (size_t)nbrow * mW * 4 : 0);
    const size_t set_bytes = off;
    const int64_t n_blocks = (n_seeds + B - 1) / B;
    // a caller that captures its stream into a graph of its own gets every kernel on that stream
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool capturing = !c->dry && hipStreamIsCapturing(s, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone;
    // two_streams 0 picks: local regions of kTwoSetMinHops hops or more alternate two blocks (their short
    // per-step FP64 kernels and the eigensolve leave most of the chip idle: +18 % at 6 and 8 hops, +13 % at
    // 16, but -3 % at 5 and -13 % at 3), everything else one block at a time with the eigensolve on the
    // second stream
    constexpr int kTwoSetMinHops = 6;
    const int tsm = c->tune.two_streams != 0 ? c->tune.two_streams : (local && c->loc >= kTwoSetMinHops ? 1 : 3);
    bool two_fit = 2.0 * (double)set_bytes <= kTwoSetBytes;
    if (two_fit && tsm == 1 && c->tune.two_streams == 0 && !c->dry && !c->ext_ws && 2 * set_bytes > c->ws_bytes) {
        // the default takes a second workspace only when the device has room for it (the current
        // workspace is given back first); else it runs one block at a time
        size_t fr = 0, tot = 0;
        two_fit = hipMemGetInfo(&fr, &tot) == hipSuccess && 2 * set_bytes + (set_bytes >> 4) <= fr + c->ws_bytes;
    }
    const int nset = n_blocks >= 2 && !c->prof && !c->in_graph && !capturing && c->es.mode == 0 &&
                             tsm == 1 &&
                             c->stream2 &&
                             two_fit
                         ? 2
                         : 1;
    off = (size_t)nset * set_bytes;
    if (!c->dry && nset == 2) c->ran_two_sets = true;
    // One block at a time (two_streams 3, or 0 when it does not pick two blocks or they do not fit): each
    // block's eigensolve runs on the second stream while the next block's sweeps run on the caller's; the
    // subspace matrix and the gathered rows alternate between two copies. Not while profiling, inside graphs
    // or for the eigen-state passes.
    const bool eig_ovl = nset == 1 && n_blocks >= 2 && !c->prof && !c->in_graph && !capturing && c->es.mode == 0 &&
                         (c->tune.two_streams == 0 || c->tune.two_streams == 3) && c->stream2;
    const size_t oH2 = take(eig_ovl ? (size_t)B * nu * nu * 8 : 0);
    const size_t oKp2 = take(eig_ovl ? (size_t)B * nu * std::max(1, c->max_row) * 8 : 0);
    const size_t oNc2 = take(eig_ovl ? (size_t)B * 4 : 0);
    const bool own_e = d_e_seed == nullptr, own_n = d_n_seed == nullptr, own_nu = d_nu_eff == nullptr;
    const size_t oE = take(own_e ? (size_t)n_seeds * 8 : 0), oN = take(own_n ? (size_t)n_seeds * 8 : 0);
    const size_t oNuOut = take(own_nu ? (size_t)n_seeds * 4 : 0);
    mar_status st = ensure_ws(c, off);
    if (st != MAR_OK) return st;
    char* w = c->ws_act;
    // profiled solve: each block's tile counts are kept for the restricted byte counts
    int32_t* plog = nullptr;
    if (sparse && c->prof && !c->dry) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
            if (n_blocks > 0 && hipMalloc((void**)&plog, (size_t)n_blocks * (nu + 1) * 4) == hipSuccess)
                c->plogs.push_back(plog);
            else plog = nullptr;
        }
    }
    auto tag = [&](bool rec, int kind, int n, int64_t blk, double dense_tiles) {
        if (!rec || !plog) return;
        ProfRec& r = c->recs.back();
        r.sp = kind;
        r.sp_n = n;
        r.sp_cnt = plog + blk * (nu + 1);
        r.sp_len = nu + 1;
        r.sp_unit = 4.0 * mar::WG * 16.0;
        r.sp_elem = (double)sizeof(T);
        r.sp_ntiles = dense_tiles;
    };
    double* e_seed = own_e ? (double*)(w + oE) : d_e_seed;
    double* n_seed = own_n ? (double*)(w + oN) : d_n_seed;
    int32_t* nu_out = own_nu ? (int32_t*)(w + oNuOut) : d_nu_eff;
    const double tau = sizeof(T) == 4 ? 1e-5 : 1e-12;
    const int64_t slab_el = stride;

    hipStream_t s_caller = s;
    if (nset == 2 && !c->dry) {   // the second stream starts after the caller's earlier work
        hipEventRecord(c->ev_fork, s_caller);
        hipStreamWaitEvent(c->stream2, c->ev_fork, 0);
    }
    for (int64_t blk0 = 0; blk0 < n_seeds; blk0 += B) {
        const int ns = (int)std::min<int64_t>(B, n_seeds - blk0);
        const int32_t* seeds = d_seeds + blk0;
        const int64_t bi = blk0 / B;
        const int set = (int)(bi % nset);
        hipStream_t s = set ? c->stream2 : s_caller;
        char* ws = w + (size_t)set * set_bytes;
        T* K = (T*)(ws + oK);
        T* Y = (T*)(ws + oY);
        T* SY = (T*)(ws + oSY);
        T* ZT = (T*)(ws + oZT);
        double* part = (double*)(ws + oPart);
        double* npart = (double*)(ws + oNP);
        double* red = (double*)(ws + oRed);
        double* redb = (double*)(ws + oRedb);
        double* h = (double*)(ws + oH);
        double* Kp = (double*)(ws + oKp);
        int32_t* nucp = (int32_t*)(ws + oNc);
        // overlapped eigensolves: odd blocks use the second copy of h and the gathered rows, and a block waits
        // until the eigensolve of the block before last has released its copy
        const int ep = (int)(bi % 2);
        if (eig_ovl && ep == 1) {
            h = (double*)(w + oH2);
            Kp = (double*)(w + oKp2);
            nucp = (int32_t*)(w + oNc2);
        }
        if (eig_ovl && bi >= 2 && !c->dry) hipStreamWaitEvent(s, c->ev_eig[ep], 0);
        double* G = (double*)(ws + oG);
        double* R = (double*)(ws + oR);
        double* C1 = (double*)(ws + oC1);
        double* BT = (double*)(ws + oBT);
        double* UU = (double*)(ws + oUU);
        double* gam = (double*)(ws + oGam);
        double* Fn = (double*)(ws + oFn);
        double* cA = (double*)(ws + oCA);
        double* cB = (double*)(ws + oCB);
        float* cAf = sizeof(T) == 4 ? (float*)(ws + oCAf) : nullptr;
        float* cBf = sizeof(T) == 4 ? (float*)(ws + oCBf) : nullptr;
        const T* cAT = sizeof(T) == 4 ? (const T*)cAf : (const T*)cA;
        const T* cBT = sizeof(T) == 4 ? (const T*)cBf : (const T*)cB;
        int32_t* active = (int32_t*)(ws + oAct);
        int32_t* nu_blk = (int32_t*)(ws + oNu);
        int32_t* sdist = (int32_t*)(ws + oDist);
        int32_t* TD = sparse ? (int32_t*)(ws + oTD) : nullptr;
        int32_t* scnt = (int32_t*)(ws + oCnt);
        int32_t* slist = (int32_t*)(ws + oList);
        int32_t* sDl = (int32_t*)(ws + oDl);
        int32_t* splan = (int32_t*)(ws + oPlan);
        uint32_t* lm0 = (uint32_t*)(ws + oM0);
        uint32_t* lm1 = (uint32_t*)(ws + oM1);
        const uint32_t* lmask = nullptr;
        if (M != c->M && bi < nset) {
            // padded rows of Y, S y and S u~ must read as zero (spmm writes rows < M only)
            launch(c, s, P_INIT, [&] { return mar::launch_zero(Y, (int64_t)slab, s); });
            launch(c, s, P_INIT, [&] { return mar::launch_zero(SY, (int64_t)slab, s); });
            launch(c, s, P_INIT, [&] { return mar::launch_zero(ZT, (int64_t)slab, s); });
        }
        launch(c, s, P_INIT, [&] {
            return mar::launch_init<T>(B, M, c->M, seeds, ns, c->diagS, nu, K, active, nu_blk, UU, s);
        });
        if (local) {
            lmask = c->loc % 2 == 0 ? lm0 : lm1;   // where the last of loc hops leaves the masks
            launch(c, s, P_SUPPORT, [&] {
                mar::launch_local_masks(c->M, nbrow, c->H.ptr, c->H.idx, seeds, ns, mW, c->loc, lm0, lm1, s);
                LaunchInfo li;
                li.wgs = 1;
                li.bytes = (double)(c->loc + 1) * (double)(nbrow + c->H.nnz) * mW * 4.0;
                return li;
            });
        }
        if (sparse) {
            // What a sweep reads beyond what this block has written must be zero. The whole-cell form gets it
            // from the update's ring of zeros and the products' row test (ring); the eigen-state passes clear
            // slabs 1.. here, and y starts at zero in both. With local regions only the tiles within one hop of
            // the regions' union are ever read, and those are cleared below.
            if (!local) {
                if (!ring)
                    launch(c, s, P_INIT, [&] {
                        return mar::launch_zero(K + slab_el, (int64_t)((size_t)(nu - 1) * stride * sizeof(T)), s);
                    });
                launch(c, s, P_INIT, [&] { return mar::launch_zero(Y, (int64_t)slab, s); });
            }
            launch(c, s, P_SUPPORT, [&] {
                return mar::launch_support(c->M, nbrow, c->H.ptr, c->H.idx, c->H.nnz, seeds, ns, (int)bpt, hsup,
                                           std::max(hsup, nu), sdist, TD, scnt, slist, sDl, s);
            });
            if (local)
                launch(c, s, P_INIT, [&] {
                    return mar::launch_zero_ring(nbrow, c->H.ptr, c->H.idx, sdist, hreach, (int)bpt, K + slab_el,
                                                 (int64_t)(stride * sizeof(T)), nu - 1, Y, nvec, s);
                });
            if (plog && !c->refused)
                hipMemcpyAsync(plog + bi * (nu + 1), scnt, (size_t)(nu + 1) * 4, hipMemcpyDeviceToDevice, s);
            // the projection plans of every step: the counts no longer change in this block
            launch(c, s, P_SUPPORT, [&] { return mar::launch_projr_plan(scnt, sDl, 0, nu, kg, target, pstride, splan, s); });
        }
        // at steps n >= 1 the dual pass also gives the norms of slab n (the unnormalized residual of step n - 1)
        if (!dual) launch(c, s, P_SPMM, [&] { return mar::launch_spmm<T>(B, c->S, K, ZT, nullptr, 0, 0, s); });
        for (int n = 0; n < nu; ++n) {
            T* Kn = K + (size_t)n * slab_el;
            const int nk = n + 1;
            const bool last = n + 1 == nu;
            int64_t swgs = 0;
            if (dual) {
                const bool rec = launch(c, s, n == 0 ? P_SPMM : P_SPMM_DOT, [&] {
                    LaunchInfo li = local && sparse
                        ? mar::launch_spmm2_list<T>(B, c->H, c->SH, Kn, Y, ZT, n == 0 ? nullptr : npart,
                                                    n == 0 ? 0 : 2, np_cap, slist, scnt, n + 1, lmask, mW,
                                                    kListWgs, s)
                        : mar::launch_spmm2<T>(B, c->H, c->SH, Kn, Y, ZT, n == 0 ? nullptr : npart, n == 0 ? 0 : 2,
                                               np_cap, s, TD, n + 1, lmask, mW, sparse ? sdist : nullptr);
                    swgs = li.wgs;
                    return li;
                });
                tag(rec, SP_FRAC, n + 1, bi, (double)ntiles);
            } else if (n >= 1) {
                launch(c, s, P_SPMM_DOT, [&] {
                    LaunchInfo li = mar::launch_spmm<T>(B, c->S, Kn, ZT, npart, 2, np_cap, s);
                    swgs = li.wgs;
                    return li;
                });
            }
            // the S-norm partials of slab n, summed across workgroups (a coalesced transposing reduction);
            // the breakdown test itself runs at the start of this step's coefficient kernel
            if (n >= 1)
                // (the projection partials of this step are not written yet: their buffer is the scratch)
                launch(c, s, P_REDUCE, [&] {
                    return mar::launch_reduce(npart, swgs, 2 * B, redb, nullptr, B, nu, n, s, part, part_cap);
                });
            if (!dual) launch(c, s, P_SPMM, [&] { return mar::launch_spmm<T>(B, c->H, Kn, Y, nullptr, 0, 0, s); });
            if (sparse) {
                const bool rec = launch(c, s, P_SPMM, [&] {
                    return local ? mar::launch_spmm_list<T>(B, c->SH, Y, SY, slist, scnt, n, lmask, mW, kListWgs, s)
                                 : mar::launch_spmm<T>(B, c->SH, Y, SY, nullptr, 0, 0, s, TD, n, lmask, mW, sdist);
                });
                tag(rec, SP_FRAC, n, bi, (double)ntiles);
                const int64_t grid = mar::projr_sp_grid(target, nk, kg);
                int32_t* plan_n = splan + (int64_t)n * pstride;
                const bool rp = launch(c, s, P_PROJR, [&] {
                    return mar::launch_projr_sp<T>(B, K, M, stride, n, ZT, SY, Y, slist, scnt, plan_n, grid, part,
                                                   part_cap, pvar, s);
                });
                tag(rp, SP_PROJR, n, bi, (double)ntiles);
                launch(c, s, P_REDUCE, [&] { return mar::launch_reduce_sp(part, plan_n, grid, kg, nk, B, red, s); });
            } else {
                launch(c, s, P_SPMM, [&] {
                    return local ? mar::launch_spmm<T>(B, c->SH, Y, SY, nullptr, 0, 0, s, nullptr, 0, lmask, mW)
                                 : mar::launch_spmm<T>(B, c->S, Y, SY, nullptr, 0, 0, s);
                });
                int64_t ngroups = 0;
                launch(c, s, P_PROJR, [&] {
                    return mar::launch_projr<T>(B, K, M, stride, nk, ZT, SY, Y, part, part_cap, &ngroups, target,
                                                pvar, s);
                });
                const int64_t L = (int64_t)3 * nk * B;
                launch(c, s, P_REDUCE, [&] { return mar::launch_reduce(part, ngroups, L, red, nullptr, B, nu, n, s); });
            }
            launch(c, s, P_COEF, [&] {
                return mar::launch_coef(B, nu, n, red, h, G, R, C1, BT, UU, cA, cB, cAf, cBf, gam, Fn, active,
                                        nu_blk, tau, n >= 1 ? redb : nullptr, s);
            });
            const bool ru = launch(c, s, P_UPD2, [&] {
                // w' goes straight into slab n + 1, unnormalized (its scale is handled by k_coef)
                T* wout = last ? nullptr : K + (size_t)(n + 1) * slab_el;
                // with support tracking the tiles are taken in distance order, one workgroup per tile (local
                // regions: a grid-stride loop over the few tiles of the regions, which stay cached)
                if (sparse) {
                    const bool nt = !local && (double)(n + 2) * (double)slab > mar::kNtSweepBytes;
                    return mar::launch_upd2_list<T>(B, K, M, stride, n, cAT, cBT, gam, Fn, Y, wout, !last, slist,
                                                    sDl, scnt, n + 1, ring ? n + 1 + kg : n + 1,
                                                    local ? kListWgs : ntiles, nt, s, upd_acc64);
                }
                return mar::launch_upd2<T>(B, K, M, stride, n, cAT, cBT, gam, Fn, Y, wout, !last, upd_q, s,
                                           upd_acc64);
            });
            tag(ru, last ? SP_UPD2_LAST : SP_UPD2, n, bi, (double)ntiles);
            if (last) break;
        }
        // rows K[P(j), :] leave the basis, then the subspace eigensolve and assembly
        launch(c, s, P_EIG, [&] {
            return mar::launch_gather<T>(B, ns, seeds, nu, nu_blk, K, stride, c->Hrp, c->Hcol, c->max_row, Kp, nucp,
                                         s);
        });
        hipStream_t se = s;
        if (eig_ovl && !c->dry) {   // the eigensolve reads only h, the gathered rows and H: off the caller's stream
            hipEventRecord(c->ev_ready[ep], s);
            hipStreamWaitEvent(c->stream2, c->ev_ready[ep], 0);
            se = c->stream2;
        }
        eig_stage<T>(c, se, B, ns, seeds, nu, h, nucp, Kp, K, stride, M, mu, kT, d_rho, e_seed + blk0, n_seed + blk0,
                     nu_out + blk0, d_eps ? d_eps + blk0 * nu : nullptr, d_w ? d_w + blk0 * nu : nullptr, blk0);
        if (eig_ovl && !c->dry) hipEventRecord(c->ev_eig[ep], c->stream2);
    }
    if ((nset == 2 || eig_ovl) && !c->dry) {   // the caller's stream waits for the second stream's work
        hipEventRecord(c->ev_join, c->stream2);
        hipStreamWaitEvent(s, c->ev_join, 0);
    }
    if (!c->zc_defer && !c->es.mode) launch(c, s, P_SUM, [&] { return mar::launch_sum(e_seed, n_seeds, d_e_band, s); });
    if (c->refused) {
        c->refused = false;
        return set_err(c, MAR_ERR_STATE, "internal error: a partial-sum buffer was too small; solve not run");
    }
    HIP_OR(c, hipGetLastError());
    return MAR_OK;
}

mar_status check_scalars(mar_ctx* c, int64_t n_seeds, int32_t nu, double mu, double kT, mar_precision prec,
                         mar_form form) {
    if (n_seeds < 0) return set_err(c, MAR_ERR_ARG, "n_seeds < 0");
    if (nu < 1 || nu > c->M) return set_err(c, MAR_ERR_ARG, fmt("nu = %d outside [1, M = %lld]", nu, (long long)c->M));
    if (!std::isfinite(mu)) return set_err(c, MAR_ERR_ARG, "mu is not finite");
    if (!(kT >= 0.0) || !std::isfinite(kT)) return set_err(c, MAR_ERR_ARG, "kT must be finite and >= 0");
    if (prec != MAR_FP64 && prec != MAR_FP32) return set_err(c, MAR_ERR_ARG, "unknown precision");
    if (form != MAR_FORM_BATCHED && form != MAR_FORM_PLAIN) return set_err(c, MAR_ERR_ARG, "unknown form");
    if (mar::eig_lds_bytes(nu, c->max_row, false) > 160 * 1024)
        return set_err(c, MAR_ERR_ARG, fmt("nu = %d too large for the subspace solver with rows of %d entries", nu,
                                           c->max_row));
    return MAR_OK;
}

// MAR_ERR_NOCONV for the first seed whose subspace eigensolve did not converge.
mar_status check_noconv(mar_ctx* c, const int32_t* seeds, const std::vector<int32_t>& nuv) {
    for (size_t i = 0; i < nuv.size(); ++i)
        if (nuv[i] == mar::NU_NOCONV)
            return set_err(c, MAR_ERR_NOCONV,
                           fmt("the subspace eigensolve of seed %d did not converge within %d Jacobi sweeps", seeds[i],
                               c->tune.eig_max_sweeps > 0 ? c->tune.eig_max_sweeps : 40));
    return MAR_OK;
}

// Validation shared by the device-side entry points.
mar_status check_request(mar_ctx* c, const mar_request& r) {
    mar_status st = check_scalars(c, r.n_seeds, r.nu, r.mu, r.kT, r.prec, r.form);
    if (st != MAR_OK) return st;
    if (!r.d_e_band) return set_err(c, MAR_ERR_ARG, "e_band output is NULL");
    if (r.n_seeds > 0 && (!r.d_seeds || !r.d_rho)) return set_err(c, MAR_ERR_ARG, "seeds or rho is NULL");
    return MAR_OK;
}

// Enqueue one solve (validated) on stream s with a resolved plan.
mar_status dispatch_solve(mar_ctx* c, const mar_request& r, const Plan& pl, hipStream_t s) {
    c->refused = false;
    if (c->loc >= 0) {
        const int vec = r.prec == MAR_FP32 ? 4 : 2;
        if (!c->H.bsr || c->SH.nnz != c->H.nnz || !pl.delayed || pl.B < vec)
            return set_err(c, MAR_ERR_ARG,
                           fmt("a local region needs a 4x4-block H and the batched delayed form with blocks of at "
                               "least %d seeds (block %d)", vec, pl.B));
    }
    mar_status st;
    if (r.prec == MAR_FP32)
        st = pl.delayed ? run_solve_delayed<float>(c, r.d_seeds, r.n_seeds, r.nu, r.mu, r.kT, pl.B, pl.variant,
                                                   r.d_rho, r.d_e_band, r.d_e_seed, r.d_n_seed, r.d_nu_eff,
                                                   r.d_eps, r.d_weight, s)
                        : run_solve<float>(c, r.d_seeds, r.n_seeds, r.nu, r.mu, r.kT, pl.B, r.d_rho, r.d_e_band,
                                           r.d_e_seed, r.d_n_seed, r.d_nu_eff, r.d_eps, r.d_weight, s);
    else
        st = pl.delayed ? run_solve_delayed<double>(c, r.d_seeds, r.n_seeds, r.nu, r.mu, r.kT, pl.B, pl.variant,
                                                    r.d_rho, r.d_e_band, r.d_e_seed, r.d_n_seed, r.d_nu_eff,
                                                    r.d_eps, r.d_weight, s)
                        : run_solve<double>(c, r.d_seeds, r.n_seeds, r.nu, r.mu, r.kT, pl.B, r.d_rho, r.d_e_band,
                                            r.d_e_seed, r.d_n_seed, r.d_nu_eff, r.d_eps, r.d_weight, s);
    return st;
}

// ------------------------------------------------------------- graph cache
// Instantiated graphs of mar_solve_many, keyed by the exact request set.
struct GraphEntry {
    std::vector<mar_ctx*> ctxs;
    std::vector<char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    std::vector<hipEvent_t> events;
    void release() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        for (auto e : events) hipEventDestroy(e);
        if (cap) hipStreamDestroy(cap);
        exec = nullptr;
        graph = nullptr;
        cap = nullptr;
        events.clear();
    }
};
std::mutex g_graph_mu;
std::vector<GraphEntry*> g_graphs;   // most recent last
constexpr size_t kMaxGraphs = 16;

void drop_graphs_of(mar_ctx* c) {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (size_t i = 0; i < g_graphs.size();) {
        GraphEntry* g = g_graphs[i];
        if (std::find(g->ctxs.begin(), g->ctxs.end(), c) != g->ctxs.end()) {
            g->release();
            delete g;
            g_graphs.erase(g_graphs.begin() + i);
        } else {
            ++i;
        }
    }
}

template <class X>
void put(std::vector<char>& k, const X& x) {
    const char* p = reinterpret_cast<const char*>(&x);
    k.insert(k.end(), p, p + sizeof(X));
}

// Field by field: padding bytes of the structs are not part of the key.
void put_request(std::vector<char>& k, mar_ctx* c, const mar_request& r, const Plan& pl) {
    put(k, c);
    put(k, r.d_seeds);
    put(k, r.n_seeds);
    put(k, r.nu);
    put(k, r.mu);
    put(k, r.kT);
    put(k, (int32_t)r.prec);
    put(k, (int32_t)r.form);
    put(k, r.d_rho);
    put(k, r.d_e_band);
    put(k, r.d_e_seed);
    put(k, r.d_n_seed);
    put(k, r.d_nu_eff);
    put(k, r.d_eps);
    put(k, r.d_weight);
    put(k, pl.B);
    put(k, (int32_t)pl.delayed);
    put(k, pl.variant);
    put(k, c->tune);
    put(k, c->loc);
    put(k, c->ws);
}

}  // namespace

// ======================================================================= ABI
extern "C" {

mar_status mar_create(int64_t M, const int64_t* H_rowptr, const int32_t* H_col, const double* H_val,
                      const int64_t* S_rowptr, const int32_t* S_col, const double* S_val, mar_ctx** out) {
    if (!out) return set_err(nullptr, MAR_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (M < 1 || M >= (int64_t)INT32_MAX) return set_err(nullptr, MAR_ERR_ARG, "M must be in [1, 2^31)");
    std::string msg;
    mar_status st;
    if ((st = check_csr(M, H_rowptr, H_col, H_val, "H", msg)) != MAR_OK) return set_err(nullptr, st, msg);
    if ((st = check_csr(M, S_rowptr, S_col, S_val, "S", msg)) != MAR_OK) return set_err(nullptr, st, msg);
    if ((st = check_sym(M, H_rowptr, H_col, H_val, "H", msg)) != MAR_OK) return set_err(nullptr, st, msg);
    if ((st = check_sym(M, S_rowptr, S_col, S_val, "S", msg)) != MAR_OK) return set_err(nullptr, st, msg);
    int max_row = 0;
    for (int64_t i = 0; i < M; ++i) max_row = std::max<int>(max_row, (int)(H_rowptr[i + 1] - H_rowptr[i]));
    if (max_row > mar::MAX_ROW)
        return set_err(nullptr, MAR_ERR_ARG, fmt("a row of H stores %d entries (at most %d supported)", max_row,
                                                 mar::MAX_ROW));
    std::vector<double> svalH(H_rowptr[M], 0.0), diag(M, 0.0);
    for (int64_t i = 0; i < M; ++i)
        for (int64_t t = S_rowptr[i]; t < S_rowptr[i + 1]; ++t) {
            const int64_t u = find_slot(H_rowptr, H_col, i, S_col[t]);
            if (u < 0)
                return set_err(nullptr, MAR_ERR_PATTERN,
                               fmt("S stores (%lld, %d) which H does not", (long long)i, S_col[t]));
            svalH[u] = S_val[t];
            if (S_col[t] == i) diag[i] = S_val[t];
        }
    for (int64_t i = 0; i < M; ++i)
        if (!(diag[i] > 0.0))
            return set_err(nullptr, MAR_ERR_NOT_SPD, fmt("S_jj = %g <= 0 at j = %lld", diag[i], (long long)i));

    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess || ndev < 1) return set_err(nullptr, MAR_ERR_HIP, "no HIP device available");
    mar_ctx* c = new mar_ctx();
    hipGetDevice(&c->device);
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        c->n_cu < 1)
        c->n_cu = 1;
    c->M = M;
    c->nnzH = H_rowptr[M];
    c->nnzS = S_rowptr[M];
    c->max_row = max_row;
    c->tune = mar_tuning{0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < MAR_PROF_CLASSES; ++k) {
        std::memset(&c->agg[k], 0, sizeof(mar_prof_entry));
        if (k < P_COUNT) std::snprintf(c->agg[k].name, sizeof c->agg[k].name, "%s", kProfNames[k]);
    }
    auto fail = [&](mar_status s2) {
        g_create_err = c->err;
        delete c;
        return s2;
    };
    if ((st = build_devmat(c, M, H_rowptr, H_col, H_val, c->H)) != MAR_OK) return fail(st);
    if ((st = build_devmat(c, M, S_rowptr, S_col, S_val, c->S)) != MAR_OK) return fail(st);
    if (c->H.bsr && (st = build_devmat(c, M, H_rowptr, H_col, svalH.data(), c->SH)) != MAR_OK) return fail(st);
    std::vector<int32_t> rp32(M + 1);
    for (int64_t i = 0; i <= M; ++i) rp32[i] = (int32_t)H_rowptr[i];
    if ((st = upload(c, &c->Hrp, rp32.data(), rp32.size())) != MAR_OK) return fail(st);
    if ((st = upload(c, &c->Hcol, H_col, (size_t)c->nnzH)) != MAR_OK) return fail(st);
    if ((st = upload(c, &c->Hval, H_val, (size_t)c->nnzH)) != MAR_OK) return fail(st);
    if ((st = upload(c, &c->SvalH, svalH.data(), svalH.size())) != MAR_OK) return fail(st);
    if ((st = upload(c, &c->diagS, diag.data(), diag.size())) != MAR_OK) return fail(st);
    he = hipStreamCreate(&c->stream);
    if (he == hipSuccess) he = hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    for (int i = 0; i < 2; ++i) {
        if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_ready[i], hipEventDisableTiming);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&c->ev_eig[i], hipEventDisableTiming);
    }
    if (he != hipSuccess) {
        c->err = fmt("stream creation failed: %s", hipGetErrorString(he));
        return fail(MAR_ERR_HIP);
    }
    *out = c;
    return MAR_OK;
}

void mar_destroy(mar_ctx* ctx) {
    if (!ctx) return;
    hipDeviceSynchronize();
    drop_graphs_of(ctx);
    delete ctx;
}

mar_status mar_solve_many(int32_t n_sys, mar_ctx* const* ctx, const mar_request* req, void* hip_stream) {
    if (n_sys < 1 || !ctx || !req) {
        if (n_sys >= 1 && ctx && ctx[0]) return set_err(ctx[0], MAR_ERR_ARG, "ctx or req is NULL");
        return MAR_ERR_ARG;
    }
    for (int i = 0; i < n_sys; ++i) {
        if (!ctx[i]) return ctx[0] ? set_err(ctx[0], MAR_ERR_ARG, fmt("ctx[%d] is NULL", i)) : MAR_ERR_STATE;
        for (int k = 0; k < i; ++k)
            if (ctx[k] == ctx[i]) return set_err(ctx[0], MAR_ERR_ARG, fmt("ctx[%d] repeats ctx[%d]", i, k));
        if (ctx[i]->device != ctx[0]->device)
            return set_err(ctx[0], MAR_ERR_ARG, fmt("ctx[%d] is on another device", i));
        mar_status st = check_request(ctx[i], req[i]);
        if (st != MAR_OK) return st;
        // Two host crashes (segmentation faults, no GPU fault) followed a graph capture on contexts whose
        // earlier solves ran two seed blocks in flight; the cause is not known, so that sequence is refused.
        if (ctx[i]->ran_two_sets)
            return set_err(ctx[i], MAR_ERR_STATE,
                           fmt("ctx[%d] has run solves with two seed blocks in flight; mar_solve_many refuses such a "
                               "context (use another context, or two_streams 3 or 2 from its creation on)", i));
    }
    mar_ctx* c0 = ctx[0];
    HIP_OR(c0, hipSetDevice(c0->device));
    std::vector<Plan> plans(n_sys);
    std::vector<char> key;
    for (int i = 0; i < n_sys; ++i) {
        plans[i] = plan_solve(ctx[i], req[i].nu, req[i].prec, req[i].form, req[i].n_seeds);
        put_request(key, ctx[i], req[i], plans[i]);
    }
    GraphEntry* hit = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (size_t g = 0; g < g_graphs.size(); ++g)
            if (g_graphs[g]->key == key) {
                hit = g_graphs[g];
                g_graphs.erase(g_graphs.begin() + g);
                g_graphs.push_back(hit);   // most recently used last
                break;
            }
    }
    if (!hit) {
        // size and allocate every workspace first: nothing may allocate under capture
        for (int i = 0; i < n_sys; ++i) {
            ctx[i]->dry = true;
            ctx[i]->in_graph = true;
            mar_status st = dispatch_solve(ctx[i], req[i], plans[i], ctx[i]->stream);
            ctx[i]->dry = false;
            ctx[i]->in_graph = false;
            if (st != MAR_OK) return st;
        }
        HIP_OR(c0, hipDeviceSynchronize());
        key.clear();   // the workspaces may have moved
        for (int i = 0; i < n_sys; ++i) put_request(key, ctx[i], req[i], plans[i]);
        auto* g = new GraphEntry();
        g->ctxs.assign(ctx, ctx + n_sys);
        g->key = key;
        auto fail = [&](mar_ctx* c, mar_status st, const std::string& m) {
            g->release();
            delete g;
            return set_err(c, st, m);
        };
        if (hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking) != hipSuccess)
            return fail(c0, MAR_ERR_HIP, "hipStreamCreateWithFlags failed");
        g->events.resize(n_sys + 1, nullptr);
        for (auto& e : g->events)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return fail(c0, MAR_ERR_HIP, "hipEventCreateWithFlags failed");
        std::vector<bool> prof(n_sys);
        for (int i = 0; i < n_sys; ++i) {
            prof[i] = ctx[i]->prof;
            ctx[i]->prof = false;   // no timing events inside a graph
        }
        hipError_t he = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
        mar_status st = MAR_OK;
        int bad = 0;
        if (he == hipSuccess) {
            // fork: every system's launch sequence is a branch off one event
            hipEventRecord(g->events[n_sys], g->cap);
            for (int i = 0; i < n_sys && st == MAR_OK; ++i) {
                hipStreamWaitEvent(ctx[i]->stream, g->events[n_sys], 0);
                ctx[i]->in_graph = true;
                st = dispatch_solve(ctx[i], req[i], plans[i], ctx[i]->stream);
                ctx[i]->in_graph = false;
                if (st != MAR_OK) bad = i;
                hipEventRecord(g->events[i], ctx[i]->stream);
                hipStreamWaitEvent(g->cap, g->events[i], 0);
            }
            he = hipStreamEndCapture(g->cap, &g->graph);
        }
        for (int i = 0; i < n_sys; ++i) ctx[i]->prof = prof[i];
        if (st != MAR_OK) {
            const std::string m = ctx[bad]->err;
            return fail(ctx[bad], st, m);
        }
        if (he != hipSuccess) return fail(c0, MAR_ERR_HIP, fmt("graph capture failed: %s", hipGetErrorString(he)));
        he = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (he != hipSuccess)
            return fail(c0, MAR_ERR_HIP, fmt("hipGraphInstantiate failed: %s", hipGetErrorString(he)));
        std::lock_guard<std::mutex> lk(g_graph_mu);
        if (g_graphs.size() >= kMaxGraphs) {
            GraphEntry* old = g_graphs.front();
            hipDeviceSynchronize();
            old->release();
            delete old;
            g_graphs.erase(g_graphs.begin());
        }
        g_graphs.push_back(g);
        hit = g;
    }
    HIP_OR(c0, hipGraphLaunch(hit->exec, (hipStream_t)hip_stream));
    return MAR_OK;
}

mar_status mar_autotune(mar_ctx* c, int32_t nu, mar_precision prec, const int32_t* d_seeds, int64_t n_seeds,
                        double mu, double kT, void* hip_stream, int32_t* best_block, int32_t* best_variant,
                        double* best_rate) {
    if (!c) return MAR_ERR_STATE;
    mar_status st = check_scalars(c, n_seeds, nu, mu, kT, prec, MAR_FORM_BATCHED);
    if (st != MAR_OK) return st;
    if (n_seeds < 1 || !d_seeds) return set_err(c, MAR_ERR_ARG, "the autotuner needs at least one seed");
    HIP_OR(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    if (!c->tune_buf) {
        void* p = nullptr;
        HIP_OR(c, hipMalloc(&p, (size_t)(c->nnzH + 1) * 8));
        c->tune_buf = (double*)p;
        c->allocs.push_back(p);
    }
    const int64_t n_probe = std::min<int64_t>(n_seeds, 256);
    mar_request r{d_seeds, n_probe, nu, mu, kT, prec, MAR_FORM_BATCHED, c->tune_buf, c->tune_buf + c->nnzH,
                  nullptr, nullptr, nullptr, nullptr, nullptr};
    const mar_tuning saved = c->tune;
    const bool delayed = saved.schedule != MAR_SCHED_TEXTBOOK;
    const int cap = std::min<int64_t>(block_cap(c, nu, prec, delayed), pow2_floor(n_probe) * 2);
    hipEvent_t e0, e1;
    HIP_OR(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return set_err(c, MAR_ERR_HIP, "hipEventCreate failed");
    }
    int bestB = 0, bestV = 0;
    double bestR = -1.0;
    int B0 = std::min(cap, 16), cap_t = cap;
    if (c->loc >= 0) {   // local regions need blocks of at least one 16-byte vector of seeds
        B0 = std::max(B0, prec == MAR_FP32 ? 4 : 2);
        cap_t = std::max(cap_t, B0);
    }
    for (int B = B0; B <= cap_t && st == MAR_OK; B *= 2) {
        for (int v : {0, 3}) {
            if (!delayed && v != 0) continue;
            Plan pl{B, delayed, v};
            st = dispatch_solve(c, r, pl, s);          // warm-up (sizes the workspace)
            if (st != MAR_OK) break;
            hipEventRecord(e0, s);
            st = dispatch_solve(c, r, pl, s);
            hipEventRecord(e1, s);
            if (st != MAR_OK) break;
            if (hipEventSynchronize(e1) != hipSuccess) {
                st = set_err(c, MAR_ERR_HIP, "autotuner: hipEventSynchronize failed");
                break;
            }
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            const double rate = ms > 0.f ? n_probe / (ms * 1e-3) : 0.0;
            if (rate > bestR) {
                bestR = rate;
                bestB = B;
                bestV = v;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != MAR_OK) return st;
    c->tuned[{nu, (int)prec}] = {bestB, bestV};
    if (best_block) *best_block = bestB;
    if (best_variant) *best_variant = bestV;
    if (best_rate) *best_rate = bestR;
    return MAR_OK;
}

mar_status mar_solve_async(mar_ctx* c, const int32_t* d_seeds, int64_t n_seeds, int32_t nu, double mu, double kT,
                           mar_precision prec, mar_form form, double* d_rho, double* d_e_band, double* d_e_seed,
                           double* d_n_seed, int32_t* d_nu_eff, double* d_eps, double* d_weight, void* hip_stream) {
    if (!c) return MAR_ERR_STATE;
    mar_status st = check_scalars(c, n_seeds, nu, mu, kT, prec, form);
    if (st != MAR_OK) return st;
    if (!d_e_band) return set_err(c, MAR_ERR_ARG, "e_band output is NULL");
    if (n_seeds > 0 && (!d_seeds || !d_rho)) return set_err(c, MAR_ERR_ARG, "seeds or rho is NULL");
    HIP_OR(c, hipSetDevice(c->device));
    mar_request r{d_seeds, n_seeds, nu, mu, kT, prec, form, d_rho, d_e_band, d_e_seed, d_n_seed, d_nu_eff, d_eps,
                  d_weight};
    return dispatch_solve(c, r, plan_solve(c, nu, prec, form, n_seeds), (hipStream_t)hip_stream);
}

mar_status mar_solve_fermi_async(mar_ctx* c, const int32_t* d_seeds, int64_t n_seeds, int32_t nu, double n_target,
                                 double kT, mar_precision prec, mar_form form, double* d_rho, double* d_e_band,
                                 double* d_e_seed, double* d_n_seed, int32_t* d_nu_eff, double* d_eps,
                                 double* d_weight, double* d_mu, void* hip_stream) {
    if (!c) return MAR_ERR_STATE;
    mar_status st = check_scalars(c, n_seeds, nu, 0.0, kT, prec, form);
    if (st != MAR_OK) return st;
    if (!std::isfinite(n_target) || n_target < 0.0) return set_err(c, MAR_ERR_ARG, "n_target must be finite and >= 0");
    if (!d_e_band || !d_mu) return set_err(c, MAR_ERR_ARG, "e_band or mu output is NULL");
    if (n_seeds > 0 && (!d_seeds || !d_rho)) return set_err(c, MAR_ERR_ARG, "seeds or rho is NULL");
    if ((size_t)nu > (size_t)mar::MAX_NU_ASSEMBLE) return set_err(c, MAR_ERR_ARG, "nu too large for the deferred assembly");
    HIP_OR(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    // levels, weights, kept eigenvector rows and per-seed results for all listed seeds
    const size_t n = (size_t)n_seeds, nl = n * nu;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t oZ = take(nl * c->max_row * 8), oEps = take(d_eps ? 0 : nl * 8), oW = take(d_weight ? 0 : nl * 8);
    const size_t oE = take(d_e_seed ? 0 : n * 8), oN = take(d_n_seed ? 0 : n * 8), oNu = take(d_nu_eff ? 0 : n * 4);
    const size_t oPart = take(2 * 512 * 8), oSt = take(4 * 8);
    if (off > c->fws_bytes) {
        if (c->fws) {
            HIP_OR(c, hipDeviceSynchronize());
            HIP_OR(c, hipFree(c->fws));
        }
        c->fws = nullptr;
        c->fws_bytes = 0;
        void* p = nullptr;
        HIP_OR(c, hipMalloc(&p, off));
        c->fws = (char*)p;
        c->fws_bytes = off;
    }
    char* f = c->fws;
    double* zc = (double*)(f + oZ);
    double* eps = d_eps ? d_eps : (double*)(f + oEps);
    double* wt = d_weight ? d_weight : (double*)(f + oW);
    double* e_seed = d_e_seed ? d_e_seed : (double*)(f + oE);
    double* n_seed = d_n_seed ? d_n_seed : (double*)(f + oN);
    int32_t* nu_eff = d_nu_eff ? d_nu_eff : (int32_t*)(f + oNu);
    double* part = (double*)(f + oPart);
    double* stt = (double*)(f + oSt);
    // 1. subspaces and eigenpairs of every seed, rows e_i.v_alpha kept
    mar_request r{d_seeds, n_seeds, nu, 0.0, kT, prec, form, d_rho, d_e_band, e_seed, n_seed, nu_eff, eps, wt};
    c->zc_defer = zc;
    st = dispatch_solve(c, r, plan_solve(c, nu, prec, form, n_seeds), s);
    c->zc_defer = nullptr;
    if (st != MAR_OK) return st;
    // 2. Fermi level by bisection on the device, 3. assembly at that level, 4. E_band
    launch(c, s, P_MU, [&] {
        return mar::launch_fermi_search(n_seeds, nu, nu_eff, eps, wt, n_target, kT, 200, part, stt, d_mu, s);
    });
    launch(c, s, P_EIG, [&] {
        return mar::launch_assemble((int)n_seeds, d_seeds, nu, nu_eff, eps, zc, c->max_row, c->Hrp, c->Hcol, c->Hval,
                                    c->SvalH, stt + 2, kT, d_rho, e_seed, n_seed, s);
    });
    launch(c, s, P_SUM, [&] { return mar::launch_sum(e_seed, n_seeds, d_e_band, s); });
    if (c->refused) {
        c->refused = false;
        return set_err(c, MAR_ERR_STATE, "internal error: a launch was refused; solve not completed");
    }
    HIP_OR(c, hipGetLastError());
    return MAR_OK;
}

mar_status mar_eigen_state_async(mar_ctx* c, const int32_t* d_seeds, int64_t n_seeds, int32_t nu, int32_t k,
                                 double sigma, mar_precision prec, mar_form form, double* d_phi, double* d_levels,
                                 int32_t* d_ref, void* hip_stream) {
    if (!c) return MAR_ERR_STATE;
    mar_status st = check_scalars(c, n_seeds, nu, 0.0, 0.0, prec, form);
    if (st != MAR_OK) return st;
    if (n_seeds < 1 || !d_seeds) return set_err(c, MAR_ERR_ARG, "eigen states need at least one seed");
    if (k < 1 || k > n_seeds) return set_err(c, MAR_ERR_ARG, fmt("k = %d outside [1, n_seeds = %lld]", k, (long long)n_seeds));
    if (!(sigma >= 0.0) || !std::isfinite(sigma)) return set_err(c, MAR_ERR_ARG, "sigma must be finite and >= 0");
    if (!d_phi || !d_levels) return set_err(c, MAR_ERR_ARG, "phi or levels output is NULL");
    if ((size_t)nu > (size_t)mar::MAX_NU_ASSEMBLE) return set_err(c, MAR_ERR_ARG, "nu too large for the eigen states");
    if (c->loc >= 0) return set_err(c, MAR_ERR_ARG, "eigen states are not available with a local region");
    HIP_OR(c, hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const Plan pl = plan_solve(c, nu, prec, form, n_seeds);
    const size_t n = (size_t)n_seeds, nl = n * nu, Mp = (size_t)(c->M + 3) / 4 * 4;
    const int groups = 64;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t oZ = take(nl * c->max_row * 8), oEps = take(nl * 8), oW = take(nl * 8), oE = take(n * 8),
                 oN = take(n * 8), oNu = take(n * 4), oPart = take(3 * 512 * 8), oSt = take(8 * 8),
                 oCm = take(n * 8), oAm = take(n * 4), oRef = take(4 * 4), oRs = take(4), oRg = take((size_t)nu * (nu + 1) * 8),
                 oY = take((size_t)nu * nu * 8), oE1 = take((size_t)nu * 8), oYr = take((size_t)nu * 8),
                 oVr = take(Mp * 8), oPd = take((size_t)groups * nu * pl.B * 8), oPr = take((size_t)nu * pl.B * 8),
                 o1 = take(4 * 8);
    if (off > c->fws_bytes) {
        if (c->fws) {
            HIP_OR(c, hipDeviceSynchronize());
            HIP_OR(c, hipFree(c->fws));
        }
        c->fws = nullptr;
        c->fws_bytes = 0;
        void* p = nullptr;
        HIP_OR(c, hipMalloc(&p, off));
        c->fws = (char*)p;
        c->fws_bytes = off;
    }
    char* f = c->fws;
    double* zc = (double*)(f + oZ);
    double* eps = (double*)(f + oEps);
    double* wt = (double*)(f + oW);
    int32_t* nu_eff = (int32_t*)(f + oNu);
    int32_t* ref = d_ref ? d_ref : (int32_t*)(f + oRef);
    int32_t* refseed = (int32_t*)(f + oRs);
    double* one = (double*)(f + o1);   // per-seed outputs of the one-seed reference solve
    // pass 1: levels, weights and rows e_i.v_alpha of every seed (Sec. 3: the Green's function of all seeds)
    mar_request r{d_seeds, n_seeds, nu, 0.0, 0.0, prec, form, nullptr, nullptr, (double*)(f + oE), (double*)(f + oN),
                  nu_eff, eps, wt};
    c->zc_defer = zc;
    st = dispatch_solve(c, r, pl, s);
    c->zc_defer = nullptr;
    if (st != MAR_OK) return st;
    // eta(k - 1), eps_k = eta(k - 1/2), eta(k) from the integrated density of states
    launch(c, s, P_MU, [&] {
        return mar::launch_dos_search(n_seeds, nu, nu_eff, eps, wt, sigma, k, 200, (double*)(f + oPart),
                                      (double*)(f + oSt), d_levels, s);
    });
    // the reference subspace eigenvector: the one contributing most to phi_k (Appendix)
    launch(c, s, P_EIG, [&] {
        return mar::launch_es_reference((int)n_seeds, d_seeds, nu, nu_eff, eps, zc, c->max_row, c->Hrp, c->Hcol,
                                        d_levels, sigma, (double*)(f + oCm), (int32_t*)(f + oAm), ref, refseed, s);
    });
    if (c->refused) {
        c->refused = false;
        return set_err(c, MAR_ERR_STATE, "internal error: a launch was refused; eigen state not computed");
    }
    // pass 1': the reference seed alone (B = 1), its eigenvector formed over all rows as v_ref
    c->es = mar_ctx::EsHook{};
    c->es.mode = 1;
    c->es.Rg = (double*)(f + oRg);
    c->es.Y = (double*)(f + oY);
    c->es.eps1 = (double*)(f + oE1);
    c->es.yref = (double*)(f + oYr);
    c->es.vref = (double*)(f + oVr);
    c->es.lv = d_levels;
    c->es.sigma = sigma;
    mar_request r1{refseed, 1, nu, 0.0, 0.0, prec, MAR_FORM_PLAIN, nullptr, nullptr, one, one + 1, (int32_t*)(one + 2),
                   nullptr, nullptr};
    st = dispatch_solve(c, r1, plan_solve(c, nu, prec, MAR_FORM_PLAIN, 1), s);
    if (st != MAR_OK) {
        c->es = mar_ctx::EsHook{};
        return st;
    }
    // pass 2: every seed again, with v_ref . v_alpha^(j) from K^T v_ref, then Eq. 3 with those signs
    c->es.mode = 2;
    c->es.pdot = (double*)(f + oPd);
    c->es.pred = (double*)(f + oPr);
    c->es.groups = groups;
    c->es.phi = d_phi;
    st = dispatch_solve(c, r, pl, s);
    c->es = mar_ctx::EsHook{};
    if (st != MAR_OK) return st;
    HIP_OR(c, hipGetLastError());
    return MAR_OK;
}

mar_status mar_eigen_state(mar_ctx* c, const int32_t* seeds, int64_t n_seeds, int32_t nu, int32_t k, double sigma,
                           mar_precision prec, mar_form form, double* phi, double* levels, int32_t* ref) {
    if (!c) return MAR_ERR_STATE;
    if (!phi || !levels) return set_err(c, MAR_ERR_ARG, "phi or levels output is NULL");
    if (n_seeds > 0 && !seeds) return set_err(c, MAR_ERR_ARG, "seeds is NULL");
    {
        std::vector<char> seen(c->M, 0);
        for (int64_t i = 0; i < n_seeds; ++i) {
            const int32_t j = seeds[i];
            if (j < 0 || j >= c->M) return set_err(c, MAR_ERR_ARG, fmt("seed %d outside [0, M)", j));
            if (seen[j]) return set_err(c, MAR_ERR_ARG, fmt("seed %d listed twice", j));
            seen[j] = 1;
        }
    }
    HIP_OR(c, hipSetDevice(c->device));
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    const size_t oSeeds = take(n_seeds * 4), oPhi = take(n_seeds * 8), oLv = take(3 * 8), oRef = take(3 * 4);
    if (off > c->io_bytes) {
        if (c->io) HIP_OR(c, hipFree(c->io));
        c->io = nullptr;
        c->io_bytes = 0;
        void* p = nullptr;
        HIP_OR(c, hipMalloc(&p, off));
        c->io = (char*)p;
        c->io_bytes = off;
    }
    char* b = c->io;
    hipStream_t s = c->stream;
    if (n_seeds > 0) HIP_OR(c, hipMemcpyAsync(b + oSeeds, seeds, n_seeds * 4, hipMemcpyHostToDevice, s));
    mar_status st = mar_eigen_state_async(c, (int32_t*)(b + oSeeds), n_seeds, nu, k, sigma, prec, form,
                                          (double*)(b + oPhi), (double*)(b + oLv), (int32_t*)(b + oRef), s);
    if (st != MAR_OK) return st;
    HIP_OR(c, hipMemcpyAsync(phi, b + oPhi, n_seeds * 8, hipMemcpyDeviceToHost, s));
    HIP_OR(c, hipMemcpyAsync(levels, b + oLv, 3 * 8, hipMemcpyDeviceToHost, s));
    if (ref) HIP_OR(c, hipMemcpyAsync(ref, b + oRef, 3 * 4, hipMemcpyDeviceToHost, s));
    HIP_OR(c, hipStreamSynchronize(s));
    return MAR_OK;
}

mar_status mar_solve_fermi(mar_ctx* c, const int32_t* seeds, int64_t n_seeds, int32_t nu, double n_target,
                           double kT, mar_precision prec, mar_form form, double* rho, double* e_band, double* mu,
                           double* e_seed, double* n_seed, int32_t* nu_eff, double* eps, double* weight) {
    if (!c) return MAR_ERR_STATE;
    mar_status st = check_scalars(c, n_seeds, nu, 0.0, kT, prec, form);
    if (st != MAR_OK) return st;
    if (!rho || !e_band || !mu) return set_err(c, MAR_ERR_ARG, "rho, e_band or mu output is NULL");
    if (n_seeds > 0 && !seeds) return set_err(c, MAR_ERR_ARG, "seeds is NULL");
    {
        std::vector<char> seen(c->M, 0);
        for (int64_t i = 0; i < n_seeds; ++i) {
            const int32_t j = seeds[i];
            if (j < 0 || j >= c->M) return set_err(c, MAR_ERR_ARG, fmt("seed %d outside [0, M)", j));
            if (seen[j]) return set_err(c, MAR_ERR_ARG, fmt("seed %d listed twice", j));
            seen[j] = 1;
        }
    }
    HIP_OR(c, hipSetDevice(c->device));
    const size_t nl = (size_t)n_seeds * nu;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    const size_t oSeeds = take(n_seeds * 4), oRho = take(c->nnzH * 8), oEb = take(8), oMu = take(8),
                 oE = take(n_seeds * 8), oN = take(n_seeds * 8), oNu = take(n_seeds * 4), oEps = take(eps ? nl * 8 : 0),
                 oW = take(weight ? nl * 8 : 0);
    if (off > c->io_bytes) {
        if (c->io) HIP_OR(c, hipFree(c->io));
        c->io = nullptr;
        c->io_bytes = 0;
        void* p = nullptr;
        HIP_OR(c, hipMalloc(&p, off));
        c->io = (char*)p;
        c->io_bytes = off;
    }
    char* b = c->io;
    hipStream_t s = c->stream;
    if (n_seeds > 0) HIP_OR(c, hipMemcpyAsync(b + oSeeds, seeds, n_seeds * 4, hipMemcpyHostToDevice, s));
    HIP_OR(c, hipMemcpyAsync(b + oRho, rho, c->nnzH * 8, hipMemcpyHostToDevice, s));
    st = mar_solve_fermi_async(c, (int32_t*)(b + oSeeds), n_seeds, nu, n_target, kT, prec, form, (double*)(b + oRho),
                               (double*)(b + oEb), (double*)(b + oE), (double*)(b + oN), (int32_t*)(b + oNu),
                               eps ? (double*)(b + oEps) : nullptr, weight ? (double*)(b + oW) : nullptr,
                               (double*)(b + oMu), s);
    if (st != MAR_OK) return st;
    std::vector<int32_t> nuv(n_seeds);
    HIP_OR(c, hipMemcpyAsync(rho, b + oRho, c->nnzH * 8, hipMemcpyDeviceToHost, s));
    HIP_OR(c, hipMemcpyAsync(e_band, b + oEb, 8, hipMemcpyDeviceToHost, s));
    HIP_OR(c, hipMemcpyAsync(mu, b + oMu, 8, hipMemcpyDeviceToHost, s));
    if (n_seeds > 0) {
        if (e_seed) HIP_OR(c, hipMemcpyAsync(e_seed, b + oE, n_seeds * 8, hipMemcpyDeviceToHost, s));
        if (n_seed) HIP_OR(c, hipMemcpyAsync(n_seed, b + oN, n_seeds * 8, hipMemcpyDeviceToHost, s));
        HIP_OR(c, hipMemcpyAsync(nuv.data(), b + oNu, n_seeds * 4, hipMemcpyDeviceToHost, s));
        if (eps) HIP_OR(c, hipMemcpyAsync(eps, b + oEps, nl * 8, hipMemcpyDeviceToHost, s));
        if (weight) HIP_OR(c, hipMemcpyAsync(weight, b + oW, nl * 8, hipMemcpyDeviceToHost, s));
    }
    HIP_OR(c, hipStreamSynchronize(s));
    for (int64_t i = 0; i < n_seeds; ++i) {
        if (nu_eff) nu_eff[i] = nuv[i];
        if (nuv[i] == -1)
            return set_err(c, MAR_ERR_NOT_SPD, fmt("w^T S w < 0 for seed %d: S is not positive definite", seeds[i]));
    }
    return check_noconv(c, seeds, nuv);
}

mar_status mar_solve(mar_ctx* c, const int32_t* seeds, int64_t n_seeds, int32_t nu, double mu, double kT,
                     mar_precision prec, mar_form form, double* rho, double* e_band, double* e_seed,
                     double* n_seed, int32_t* nu_eff, double* eps, double* weight) {
    if (!c) return MAR_ERR_STATE;
    mar_status st = check_scalars(c, n_seeds, nu, mu, kT, prec, form);
    if (st != MAR_OK) return st;
    if (!rho || !e_band) return set_err(c, MAR_ERR_ARG, "rho or e_band output is NULL");
    if (n_seeds > 0 && !seeds) return set_err(c, MAR_ERR_ARG, "seeds is NULL");
    {
        std::vector<char> seen(c->M, 0);
        for (int64_t i = 0; i < n_seeds; ++i) {
            const int32_t j = seeds[i];
            if (j < 0 || j >= c->M) return set_err(c, MAR_ERR_ARG, fmt("seed %d outside [0, M)", j));
            if (seen[j]) return set_err(c, MAR_ERR_ARG, fmt("seed %d listed twice", j));
            seen[j] = 1;
        }
    }
    HIP_OR(c, hipSetDevice(c->device));
    const size_t nl = (size_t)n_seeds * nu;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align_up(b);
        return o;
    };
    const size_t oSeeds = take(n_seeds * 4), oRho = take(c->nnzH * 8), oEb = take(8), oE = take(n_seeds * 8),
                 oN = take(n_seeds * 8), oNu = take(n_seeds * 4), oEps = take(eps ? nl * 8 : 0),
                 oW = take(weight ? nl * 8 : 0);
    if (off > c->io_bytes) {
        if (c->io) HIP_OR(c, hipFree(c->io));
        c->io = nullptr;
        c->io_bytes = 0;
        void* p = nullptr;
        HIP_OR(c, hipMalloc(&p, off));
        c->io = (char*)p;
        c->io_bytes = off;
    }
    char* b = c->io;
    hipStream_t s = c->stream;
    if (n_seeds > 0) HIP_OR(c, hipMemcpyAsync(b + oSeeds, seeds, n_seeds * 4, hipMemcpyHostToDevice, s));
    HIP_OR(c, hipMemcpyAsync(b + oRho, rho, c->nnzH * 8, hipMemcpyHostToDevice, s));
    st = mar_solve_async(c, (int32_t*)(b + oSeeds), n_seeds, nu, mu, kT, prec, form, (double*)(b + oRho),
                         (double*)(b + oEb), (double*)(b + oE), (double*)(b + oN), (int32_t*)(b + oNu),
                         eps ? (double*)(b + oEps) : nullptr, weight ? (double*)(b + oW) : nullptr, s);
    if (st != MAR_OK) return st;
    std::vector<int32_t> nuv(n_seeds);
    HIP_OR(c, hipMemcpyAsync(rho, b + oRho, c->nnzH * 8, hipMemcpyDeviceToHost, s));
    HIP_OR(c, hipMemcpyAsync(e_band, b + oEb, 8, hipMemcpyDeviceToHost, s));
    if (n_seeds > 0) {
        if (e_seed) HIP_OR(c, hipMemcpyAsync(e_seed, b + oE, n_seeds * 8, hipMemcpyDeviceToHost, s));
        if (n_seed) HIP_OR(c, hipMemcpyAsync(n_seed, b + oN, n_seeds * 8, hipMemcpyDeviceToHost, s));
        HIP_OR(c, hipMemcpyAsync(nuv.data(), b + oNu, n_seeds * 4, hipMemcpyDeviceToHost, s));
        if (eps) HIP_OR(c, hipMemcpyAsync(eps, b + oEps, nl * 8, hipMemcpyDeviceToHost, s));
        if (weight) HIP_OR(c, hipMemcpyAsync(weight, b + oW, nl * 8, hipMemcpyDeviceToHost, s));
    }
    HIP_OR(c, hipStreamSynchronize(s));
    if (nu_eff && n_seeds > 0) std::memcpy(nu_eff, nuv.data(), n_seeds * 4);
    for (int64_t i = 0; i < n_seeds; ++i)
        if (nuv[i] == -1)
            return set_err(c, MAR_ERR_NOT_SPD, fmt("w^T S w < 0 for seed %d: S is not positive definite", seeds[i]));
    return check_noconv(c, seeds, nuv);
}

// Greedy distance-2 colouring of H's rows in index order: row l takes the
// smallest colour not used by an earlier row within two hops of it.
mar_status build_colouring(mar_ctx* c) {
    const int64_t M = c->M;
    std::vector<int32_t> rp(M + 1), col((size_t)c->nnzH);
    HIP_OR(c, hipMemcpy(rp.data(), c->Hrp, rp.size() * 4, hipMemcpyDeviceToHost));
    HIP_OR(c, hipMemcpy(col.data(), c->Hcol, col.size() * 4, hipMemcpyDeviceToHost));
    std::vector<int32_t> colour(M, -1);
    std::vector<int64_t> stamp;
    int ncol = 0;
    for (int64_t l = 0; l < M; ++l) {
        auto mark = [&](int64_t m) {
            if (m < l) stamp[colour[m]] = l;
        };
        for (int q = rp[l]; q < rp[l + 1]; ++q) {
            const int64_t j = col[q];
            if (stamp.size() < (size_t)ncol + 1) stamp.resize((size_t)ncol + 1, -1);
            mark(j);
            for (int t = rp[j]; t < rp[j + 1]; ++t) mark(col[t]);
        }
        if (stamp.size() < (size_t)ncol + 1) stamp.resize((size_t)ncol + 1, -1);
        int k = 0;
        while (k < ncol && stamp[k] == l) ++k;
        colour[l] = k;
        if (k == ncol) ++ncol;
    }
    std::vector<int32_t> off(ncol + 1, 0), rows(M);
    for (int64_t l = 0; l < M; ++l) ++off[colour[l] + 1];
    for (int k = 0; k < ncol; ++k) off[k + 1] += off[k];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int64_t l = 0; l < M; ++l) rows[fill[colour[l]]++] = (int32_t)l;
    mar_status st;
    if ((st = upload(c, &c->fl_coff, off.data(), off.size())) != MAR_OK) return st;
    if ((st = upload(c, &c->fl_crow, rows.data(), rows.size())) != MAR_OK) return st;
    c->fl_ncol = ncol;
    return MAR_OK;
}

mar_status mar_local_flip(mar_ctx* c, double* d_phi, double eps, const double* d_phi_ref, double cpen,
                          int32_t max_sweeps, double* d_R, int32_t* d_info, void* hip_stream) {
    if (!c) return MAR_ERR_STATE;
    if (!d_phi) return set_err(c, MAR_ERR_ARG, "phi is NULL");
    if (!std::isfinite(eps)) return set_err(c, MAR_ERR_ARG, "eps is not finite");
    if (!(cpen >= 0.0) || !std::isfinite(cpen)) return set_err(c, MAR_ERR_ARG, "c must be finite and >= 0");
    if (max_sweeps < 0) return set_err(c, MAR_ERR_ARG, "max_sweeps < 0");
    HIP_OR(c, hipSetDevice(c->device));
    if (!c->fl_crow) {
        mar_status st = build_colouring(c);
        if (st != MAR_OK) return st;
    }
    if (!c->flws) {
        void* p = nullptr;
        HIP_OR(c, hipMalloc(&p, (size_t)c->M * 25 + 16));
        c->flws = (char*)p;
    }
    double* r = (double*)c->flws;       // residual (H - eps S) phi
    double* sv = r + c->M;              // S phi_ref
    double* drr = sv + c->M;            // per colour entry: |r|^2 change of its single flip
    int8_t* flag = (int8_t*)(drr + c->M);
    mar::launch_flip(c->M, c->Hrp, c->Hcol, c->Hval, c->SvalH, eps, d_phi, d_phi_ref, cpen, c->fl_ncol, c->fl_coff,
                     c->fl_crow, max_sweeps, r, sv, drr, flag, d_R, d_info, (hipStream_t)hip_stream);
    HIP_OR(c, hipGetLastError());
    return MAR_OK;
}

int32_t mar_flip_colours(mar_ctx* c) {
    if (!c) return -1;
    if (!c->fl_crow && (hipSetDevice(c->device) != hipSuccess || build_colouring(c) != MAR_OK)) return -1;
    return c->fl_ncol;
}

mar_status mar_set_local_region(mar_ctx* c, int32_t hops) {
    if (!c) return MAR_ERR_STATE;
    if (hops >= 0 && (!c->H.bsr || c->SH.nnz != c->H.nnz))
        return set_err(c, MAR_ERR_ARG, "a local region needs H with 4x4 block structure");
    c->loc = hops < 0 ? -1 : hops;
    return MAR_OK;
}

int32_t mar_local_region(const mar_ctx* c) { return c ? c->loc : -1; }

mar_status mar_set_tuning(mar_ctx* c, const mar_tuning* t) {
    if (!c) return MAR_ERR_STATE;
    if (!t) {
        c->tune = mar_tuning{0, 0, 0, 0, 0, 0, 0, 0, 0};
        return MAR_OK;
    }
    if (t->seed_block < 0 || t->seed_block > 256 || (t->seed_block & (t->seed_block - 1)) != 0)
        return set_err(c, MAR_ERR_ARG, "seed_block must be 0 or a power of two <= 256");
    if (t->schedule < MAR_SCHED_AUTO || t->schedule > MAR_SCHED_DELAYED)
        return set_err(c, MAR_ERR_ARG, "unknown schedule");
    if (t->proj_wgs < 0) return set_err(c, MAR_ERR_ARG, "proj_wgs < 0");
    if (t->slab_pad_kb < 0 || t->slab_pad_kb > 65536) return set_err(c, MAR_ERR_ARG, "slab_pad_kb outside [0, 65536]");
    if (t->proj_variant < 0 || t->proj_variant > 7) return set_err(c, MAR_ERR_ARG, "proj_variant outside [0, 7]");
    if (t->upd_q != 0 && t->upd_q != 2 && t->upd_q != 4 && t->upd_q != 8)
        return set_err(c, MAR_ERR_ARG, "upd_q must be 0, 2, 4 or 8");
    if (t->support_off != 0 && t->support_off != 1) return set_err(c, MAR_ERR_ARG, "support_off must be 0 or 1");
    if (t->two_streams < 0 || t->two_streams > 3) return set_err(c, MAR_ERR_ARG, "two_streams must be 0, 1, 2 or 3");
    if (t->eig_max_sweeps < 0) return set_err(c, MAR_ERR_ARG, "eig_max_sweeps < 0");
    c->tune = *t;
    return MAR_OK;
}

mar_status mar_get_tuning(const mar_ctx* c, mar_tuning* t) {
    if (!c) return MAR_ERR_STATE;
    if (!t) return MAR_ERR_ARG;
    *t = c->tune;
    return MAR_OK;
}

int32_t mar_seed_block(const mar_ctx* c, int32_t nu, mar_precision prec) {
    if (!c) return 0;
    return plan_solve(c, nu, prec, MAR_FORM_BATCHED, 0).B;
}

const char* mar_last_error(const mar_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

mar_status mar_profile_enable(mar_ctx* c, int32_t on) {
    if (!c) return MAR_ERR_STATE;
    c->prof = on != 0;
    return MAR_OK;
}

mar_status mar_profile_reset(mar_ctx* c) {
    if (!c) return MAR_ERR_STATE;
    HIP_OR(c, hipDeviceSynchronize());
    for (auto& r : c->recs) {
        c->evfree.push_back(r.a);
        c->evfree.push_back(r.b);
    }
    c->recs.clear();
    for (void* p : c->plogs) hipFree(p);
    c->plogs.clear();
    for (int k = 0; k < MAR_PROF_CLASSES; ++k) {
        c->agg[k].launches = 0;
        c->agg[k].ms = c->agg[k].bytes = c->agg[k].flops = 0.0;
    }
    return MAR_OK;
}

mar_status mar_profile_collect(mar_ctx* c, mar_prof_entry* out, int32_t* n_out) {
    if (!c) return MAR_ERR_STATE;
    std::map<const int32_t*, std::vector<int32_t>> counts;   // tile counts of each logged block
    for (auto& r : c->recs) {
        HIP_OR(c, hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_OR(c, hipEventElapsedTime(&ms, r.a, r.b));
        if (r.sp != SP_NONE) {
            auto it = counts.find(r.sp_cnt);
            if (it == counts.end()) {
                std::vector<int32_t> h((size_t)r.sp_len);
                HIP_OR(c, hipMemcpy(h.data(), r.sp_cnt, h.size() * 4, hipMemcpyDeviceToHost));
                it = counts.emplace(r.sp_cnt, std::move(h)).first;
            }
            support_figures(r, it->second);
        }
        mar_prof_entry& e = c->agg[r.cls];
        e.launches += 1;
        e.ms += ms;
        e.bytes += r.bytes;
        e.flops += r.flops;
        c->evfree.push_back(r.a);
        c->evfree.push_back(r.b);
    }
    c->recs.clear();
    for (void* p : c->plogs) hipFree(p);
    c->plogs.clear();
    if (out) std::memcpy(out, c->agg, sizeof(mar_prof_entry) * MAR_PROF_CLASSES);
    if (n_out) *n_out = P_COUNT;
    return MAR_OK;
}

#ifndef MAR_BUILD_ID
#define MAR_BUILD_ID "unknown"
#endif
const char* mar_build_id(void) { return MAR_BUILD_ID; }

int32_t mar_ctx_info(const mar_ctx* c, int64_t* M, int64_t* nnz_H, int64_t* nnz_S) {
    if (!c) return -1;
    if (M) *M = c->M;
    if (nnz_H) *nnz_H = c->nnzH;
    if (nnz_S) *nnz_S = c->nnzS;
    return (c->H.bsr ? 1 : 0) | (c->S.bsr ? 2 : 0);
}

}  // extern "C"

// --------------------------------------------------- solve on a caller's workspace
namespace mar {

int ctx_device(const mar_ctx* c) { return c ? c->device : -1; }

mar_status ctx_error(mar_ctx* c, mar_status st, const char* msg) { return set_err(c, st, msg); }

// mar_solve_async on the workspace ws[0, ws_bytes) instead of the context's own:
// nothing is allocated on the device. With the batched form and no block size
// fixed by the tuning, the planned seed block is halved until the solve's
// workspace fits (a dry run sizes it); per-kernel timing is suspended for the
// call (its events and tile logs would be created on demand).
mar_status solve_async_ext(mar_ctx* c, const int32_t* d_seeds, int64_t n_seeds, int32_t nu, double mu, double kT,
                           mar_precision prec, mar_form form, double* d_rho, double* d_e_band, double* d_e_seed,
                           double* d_n_seed, int32_t* d_nu_eff, double* d_eps, double* d_weight, void* ws,
                           size_t ws_bytes, void* hip_stream) {
    if (!c) return MAR_ERR_STATE;
    mar_status st = check_scalars(c, n_seeds, nu, mu, kT, prec, form);
    if (st != MAR_OK) return st;
    if (!d_e_band) return set_err(c, MAR_ERR_ARG, "e_band output is NULL");
    if (n_seeds > 0 && (!d_seeds || !d_rho)) return set_err(c, MAR_ERR_ARG, "seeds or rho is NULL");
    if (!ws) return set_err(c, MAR_ERR_STATE, "no workspace");
    HIP_OR(c, hipSetDevice(c->device));
    const mar_request r{d_seeds, n_seeds, nu, mu, kT, prec, form, d_rho, d_e_band, d_e_seed, d_n_seed, d_nu_eff,
                        d_eps, d_weight};
    hipStream_t s = (hipStream_t)hip_stream;
    Plan pl = plan_solve(c, nu, prec, form, n_seeds);
    const int min_b = c->loc >= 0 ? (prec == MAR_FP32 ? 4 : 2) : 1;
    const bool shrink = form == MAR_FORM_BATCHED && c->tune.seed_block == 0;
    const bool prof = c->prof;
    c->prof = false;
    c->ext_ws = (char*)ws;
    c->ext_bytes = ws_bytes;
    for (;;) {
        c->ext_short = false;
        c->dry = true;
        st = dispatch_solve(c, r, pl, s);
        c->dry = false;
        if (st == MAR_OK || !c->ext_short || !shrink || pl.B / 2 < min_b) break;
        pl.B /= 2;
    }
    if (st == MAR_OK) st = dispatch_solve(c, r, pl, s);
    c->ext_ws = nullptr;
    c->ext_bytes = 0;
    c->ext_short = false;
    c->ws_act = c->ws;
    c->prof = prof;
    return st;
}

}  // namespace mar
