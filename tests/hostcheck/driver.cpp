// Drives the library's host code against the stub runtime (hip_stub.cpp) under the host sanitizers, for
// tests/test_host_sanitizer.py; test infrastructure. Kernels do not run, so every result is meaningless:
// what is checked is the host side (allocation, copies, streams, events, graph capture and its caches).
//
// Usage: driver DIR [mode]. DIR holds sys_0.bin .. sys_3.bin (M, nnz(H), nnz(S) as int64, then the CSR
// arrays of H and S). Mode 0 runs the sequence that preceded the host crashes of the multi-system path on
// the GPU: autotune and eager solves with two seed blocks in flight, then mar_solve_many on the same
// contexts (four calls: repeated requests, new seed pointers, new shapes), then the other entry points and
// mar_destroy. Mode 1 does the same with one block at a time and the eigensolves on the second stream.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "mar.h"

extern "C" long hip_stub_launches();
extern "C" long hip_stub_errors();
extern "C" size_t hip_stub_live_allocs();
extern "C" void hip_stub_report();

namespace {

struct Sys {
    int64_t M = 0, nnzH = 0, nnzS = 0;
    std::vector<int64_t> hp, sp;
    std::vector<int32_t> hc, sc;
    std::vector<double> hv, sv;
};

Sys load(const std::string& path) {
    Sys s;
    FILE* f = fopen(path.c_str(), "rb");
    if (!f) {
        perror(path.c_str());
        exit(2);
    }
    int64_t h[3];
    bool ok = fread(h, 8, 3, f) == 3;
    s.M = h[0];
    s.nnzH = h[1];
    s.nnzS = h[2];
    s.hp.resize(s.M + 1);
    s.hc.resize(s.nnzH);
    s.hv.resize(s.nnzH);
    s.sp.resize(s.M + 1);
    s.sc.resize(s.nnzS);
    s.sv.resize(s.nnzS);
    ok = ok && fread(s.hp.data(), 8, s.M + 1, f) == (size_t)(s.M + 1) &&
         fread(s.hc.data(), 4, s.nnzH, f) == (size_t)s.nnzH && fread(s.hv.data(), 8, s.nnzH, f) == (size_t)s.nnzH &&
         fread(s.sp.data(), 8, s.M + 1, f) == (size_t)(s.M + 1) &&
         fread(s.sc.data(), 4, s.nnzS, f) == (size_t)s.nnzS && fread(s.sv.data(), 8, s.nnzS, f) == (size_t)s.nnzS;
    fclose(f);
    if (!ok) {
        fprintf(stderr, "short read: %s\n", path.c_str());
        exit(2);
    }
    return s;
}

int failures = 0;
void check(mar_status st, const char* what, const mar_ctx* c) {
    if (st != MAR_OK) {
        ++failures;
        printf("  %s -> %d (%s)\n", what, (int)st, mar_last_error(c));
    }
}
#define CHECK(c, x) check((x), #x, (c))

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) {
        fprintf(stderr, "usage: driver DIR [mode]\n");
        return 2;
    }
    const std::string dir = argv[1];
    const int mode = argc > 2 ? atoi(argv[2]) : 0;
    const int nus[4] = {30, 100, 30, 100};
    Sys sys[4];
    mar_ctx* ctx[4];
    for (int i = 0; i < 4; ++i) {
        sys[i] = load(dir + "/sys_" + std::to_string(i) + ".bin");
        CHECK(nullptr, mar_create(sys[i].M, sys[i].hp.data(), sys[i].hc.data(), sys[i].hv.data(), sys[i].sp.data(),
                                  sys[i].sc.data(), sys[i].sv.data(), &ctx[i]));
    }
    hipStream_t st;
    (void)hipStreamCreate(&st);
    std::vector<int32_t*> dseeds(4), dnu(4);
    std::vector<double*> drho(4), deb(4), des(4), dns(4), deps(4), dw(4);
    for (int i = 0; i < 4; ++i) {
        std::vector<int32_t> seeds(sys[i].M);
        for (int64_t j = 0; j < sys[i].M; ++j) seeds[j] = (int32_t)j;
        (void)hipMalloc((void**)&dseeds[i], 4 * sys[i].M);
        (void)hipMemcpy(dseeds[i], seeds.data(), 4 * sys[i].M, hipMemcpyHostToDevice);
        (void)hipMalloc((void**)&drho[i], 8 * sys[i].nnzH);
        (void)hipMalloc((void**)&deb[i], 8);
        (void)hipMalloc((void**)&des[i], 8 * sys[i].M);
        (void)hipMalloc((void**)&dns[i], 8 * sys[i].M);
        (void)hipMalloc((void**)&dnu[i], 4 * sys[i].M);
        (void)hipMalloc((void**)&deps[i], 8 * sys[i].M * nus[i]);
        (void)hipMalloc((void**)&dw[i], 8 * sys[i].M * nus[i]);
    }
    printf("phase 1: autotune and eager solves (%s)\n", mode == 0 ? "two seed blocks in flight" : "one block");
    for (int i = 0; i < 4; ++i) {
        mar_tuning t;
        memset(&t, 0, sizeof t);
        t.two_streams = mode == 0 ? 1 : 3;
        if (i == 2) CHECK(ctx[i], mar_set_local_region(ctx[i], 6));
        CHECK(ctx[i], mar_set_tuning(ctx[i], &t));
        int32_t bb = 0, bv = 0;
        double br = 0;
        CHECK(ctx[i], mar_autotune(ctx[i], nus[i], MAR_FP32, dseeds[i], sys[i].M, -0.45, 0.1, st, &bb, &bv, &br));
        CHECK(ctx[i], mar_solve_async(ctx[i], dseeds[i], sys[i].M, nus[i], -0.45, 0.1, MAR_FP32, MAR_FORM_BATCHED,
                                      drho[i], deb[i], des[i], dns[i], dnu[i], deps[i], dw[i], st));
    }
    printf("phase 2: graphs over the same contexts\n");
    for (int rep = 0; rep < 4; ++rep) {
        std::vector<mar_request> req(4);
        for (int i = 0; i < 4; ++i) {
            mar_request& r = req[i];
            memset(&r, 0, sizeof r);
            const int64_t n = rep < 2 ? sys[i].M / 8 : sys[i].M / 4;   // a new shape from the third call on
            r.d_seeds = dseeds[i] + (rep % 2) * n;                      // new seed pointers every other call
            r.n_seeds = n;
            r.nu = rep == 3 ? nus[i] / 2 : nus[i];
            r.mu = -0.45;
            r.kT = 0.1;
            r.prec = MAR_FP32;
            r.form = MAR_FORM_BATCHED;
            r.d_rho = drho[i];
            r.d_e_band = deb[i];
            r.d_e_seed = des[i];
            r.d_n_seed = dns[i];
            r.d_nu_eff = dnu[i];
            r.d_eps = deps[i];
            r.d_weight = dw[i];
        }
        CHECK(ctx[0], mar_solve_many(4, ctx, req.data(), st));
        CHECK(ctx[0], mar_solve_many(4, ctx, req.data(), st));   // replay of the cached graph
    }
    printf("phase 3: host entry points and the other forms\n");
    {
        mar_ctx* c = ctx[0];
        const int n = 40;
        std::vector<int32_t> seeds(n);
        for (int j = 0; j < n; ++j) seeds[j] = 3 * j;
        std::vector<double> rho(sys[0].nnzH), es(n), ns(n), eps(n * 24), w(n * 24), phi(n), lv(3);
        std::vector<int32_t> nue(n), ref(3);
        double eb = 0, mu = 0;
        mar_tuning t;
        memset(&t, 0, sizeof t);
        CHECK(c, mar_set_tuning(c, &t));
        CHECK(c, mar_solve(c, seeds.data(), n, 24, -0.4, 0.1, MAR_FP64, MAR_FORM_PLAIN, rho.data(), &eb, es.data(),
                           ns.data(), nue.data(), eps.data(), w.data()));
        CHECK(c, mar_solve(c, seeds.data(), n, 24, -0.4, 0.1, MAR_FP32, MAR_FORM_BATCHED, rho.data(), &eb, es.data(),
                           ns.data(), nue.data(), eps.data(), w.data()));
        CHECK(c, mar_solve_fermi(c, seeds.data(), n, 24, (double)n, 0.1, MAR_FP32, MAR_FORM_BATCHED, rho.data(), &eb,
                                 &mu, es.data(), ns.data(), nue.data(), eps.data(), w.data()));
        CHECK(c, mar_eigen_state(c, seeds.data(), n, 24, 5, 0.01, MAR_FP64, MAR_FORM_BATCHED, phi.data(), lv.data(),
                                 ref.data()));
        double *dphi, *dR;
        int32_t* dinfo;
        (void)hipMalloc((void**)&dphi, 8 * sys[0].M);
        (void)hipMalloc((void**)&dR, 8 * 11);
        (void)hipMalloc((void**)&dinfo, 8);
        CHECK(c, mar_local_flip(c, dphi, -0.3, dphi, 5.0, 10, dR, dinfo, st));
        if (mar_flip_colours(c) <= 0) ++failures;
        CHECK(c, mar_solve_async_noalloc(c, dseeds[0], sys[0].M, 24, -0.4, 0.1, MAR_FP32, MAR_FORM_BATCHED, drho[0],
                                         deb[0], des[0], dns[0], dnu[0], deps[0], dw[0], st));
        CHECK(c, mar_solve_async_noalloc(c, dseeds[0], 64, 12, -0.4, 0.1, MAR_FP64, MAR_FORM_BATCHED, drho[0], deb[0],
                                         des[0], dns[0], dnu[0], deps[0], dw[0], st));
        t.two_streams = 2;
        CHECK(c, mar_set_tuning(c, &t));
        CHECK(c, mar_solve_async(c, dseeds[0], sys[0].M, 30, -0.45, 0.1, MAR_FP64, MAR_FORM_BATCHED, drho[0], deb[0],
                                 des[0], dns[0], dnu[0], deps[0], dw[0], st));
        CHECK(c, mar_set_tuning(c, nullptr));
        CHECK(c, mar_profile_enable(c, 1));
        CHECK(c, mar_solve_async(c, dseeds[0], sys[0].M, 30, -0.45, 0.1, MAR_FP32, MAR_FORM_BATCHED, drho[0], deb[0],
                                 des[0], dns[0], dnu[0], deps[0], dw[0], st));
        CHECK(c, mar_profile_enable(c, 0));
        (void)hipFree(dphi);
        (void)hipFree(dR);
        (void)hipFree(dinfo);
    }
    printf("phase 4: destroy\n");
    for (int i = 0; i < 4; ++i) mar_destroy(ctx[i]);
    for (int i = 0; i < 4; ++i) {
        (void)hipFree(dseeds[i]);
        (void)hipFree(drho[i]);
        (void)hipFree(deb[i]);
        (void)hipFree(des[i]);
        (void)hipFree(dns[i]);
        (void)hipFree(dnu[i]);
        (void)hipFree(deps[i]);
        (void)hipFree(dw[i]);
    }
    (void)hipStreamDestroy(st);
    hip_stub_report();
    // one allocation stays: the stand-in for the no-allocation entry point's static device array
    printf("done: %ld kernel launches, %ld call failures, %ld stub errors, %zu live allocations\n",
           hip_stub_launches(), (long)failures, hip_stub_errors(), hip_stub_live_allocs());
    return failures || hip_stub_errors() || hip_stub_live_allocs() > 1 ? 1 : 0;
}
