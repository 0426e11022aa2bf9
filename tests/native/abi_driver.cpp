// Driver for the host sanitizer build of the C ABI's argument validation (test
// infrastructure, run by tests/test_sanitizers.py): every entry point is
// called with arguments that must be refused before any device work, so the
// program needs no GPU.  Exit status 0 when every call returned the documented
// negative code.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "rpmfft.h"
#include "rpmfno.h"

static int fails = 0;
static void expect(int got, int want, const char* what)
{
    if (got != want) {
        std::printf("%s: got %d want %d\n", what, got, want);
        ++fails;
    }
}

int main()
{
    rpm_options o;
    rpm_default_options(&o);
    double lame[2] = {1.0, 1.0};
    rpm_problem pr;
    std::memset(&pr, 0, sizeof(pr));
    pr.n[0] = 8;
    pr.n[1] = 8;
    pr.n[2] = 8;
    pr.phase = reinterpret_cast<const uint8_t*>(0x1000);  // never dereferenced
    pr.n_phases = 1;
    pr.lame = lame;
    pr.lame0[0] = 1.0;
    pr.lame0[1] = 1.0;
    double E[6] = {0.01, 0, 0, 0, 0, 0};
    size_t bytes = 0;
    expect(rpm_workspace_size(pr.n, &o, &bytes), RPM_OK, "workspace size");
    rpm_options bad = o;
    bad.tol = -1.0;
    expect(rpm_fft_solve(&pr, E, &bad, nullptr, nullptr, nullptr, nullptr, nullptr, (void*)0x2000, 1ull << 40,
                         nullptr),
           RPM_E_INVALID, "solve tol");
    bad = o;
    bad.p_max = 65;
    expect(rpm_fft_solve(&pr, E, &bad, nullptr, nullptr, nullptr, nullptr, nullptr, (void*)0x2000, 1ull << 40,
                         nullptr),
           RPM_E_INVALID, "solve p_max");
    bad = o;
    bad.batch_cases = 3;
    expect(rpm_fft_effective_tensor(&pr, &bad, E, nullptr, (void*)0x2000, 1ull << 40, nullptr), RPM_E_INVALID,
           "eff batch");
    bad = o;
    bad.graph = 2;
    expect(rpm_fft_solve(&pr, E, &bad, nullptr, nullptr, nullptr, nullptr, nullptr, (void*)0x2000, 1ull << 40,
                         nullptr),
           RPM_E_INVALID, "graph flag");
    double Enan[6] = {NAN, 0, 0, 0, 0, 0};
    expect(rpm_fft_solve(&pr, Enan, &o, nullptr, nullptr, nullptr, nullptr, nullptr, (void*)0x2000, 1ull << 40,
                         nullptr),
           RPM_E_INVALID, "solve nan E");
    rpm_problem odd = pr;
    odd.n[0] = 7;
    expect(rpm_fft_solve(&odd, E, &o, nullptr, nullptr, nullptr, nullptr, nullptr, (void*)0x2000, 1ull << 40,
                         nullptr),
           RPM_E_UNSUPPORTED_SIZE, "solve size");
    expect(rpm_fft_solve(&pr, E, &o, nullptr, nullptr, nullptr, nullptr, nullptr, (void*)0x2000, 16, nullptr),
           RPM_E_WORKSPACE, "solve workspace");
    expect(rpm_fft_apply(&pr, E, &o, (void*)0x3000, (void*)0x3000, nullptr, nullptr, (void*)0x2000, 1ull << 40,
                         nullptr),
           RPM_E_INVALID, "apply alias");
    rpm_problem big = pr;
    big.n[0] = big.n[1] = big.n[2] = 256;
    expect(rpm_fft_apply_static(&big, E, &o, (void*)0x3000, (void*)0x4000, nullptr, nullptr, nullptr), RPM_E_SCRATCH,
           "apply static size");
    expect(rpm_fft_seed_basis(&pr, &o, nullptr, 2, nullptr, (void*)0x2000, 1ull << 40, nullptr), RPM_E_INVALID,
           "seed null");
    double S[6] = {0, 0, 0.01, 0, 0, 0};
    bad = o;
    bad.kappa = 2.0;
    expect(rpm_fft_solve_stress(&pr, S, &bad, nullptr, nullptr, nullptr, nullptr, nullptr, (void*)0x2000, 1ull << 40,
                                nullptr),
           RPM_E_INVALID, "stress kappa");
    double lam = 0, mu = 0;
    expect(rpm_lame_from_young(1.0, 0.5, &lam, &mu), RPM_E_INVALID, "lame nu");
    int32_t p = 0;
    expect(rpm_workspace_h(nullptr, 0, nullptr, 1, &p, nullptr), RPM_E_INVALID, "workspace h");
    rpm_fno_config cfg = {2, 36, 0, 4, 12};
    int64_t cnt = 0;
    expect(rpm_fno_param_count(&cfg, &cnt), RPM_E_INVALID, "fno width");
    cfg.width = 8;
    expect(rpm_fno_param_count(&cfg, &cnt), RPM_OK, "fno count");
    int32_t g[3] = {8, 8, 0};
    expect(rpm_fno_workspace_size(&cfg, g, 1, &bytes), RPM_E_INVALID, "fno grid");
    int64_t st[3] = {0, 1, 1};
    expect(rpm_gemm_bf16(0, 4, 4, 1, (const float*)0x10, st, (const float*)0x10, st, (float*)0x10, st, 1.f, 0.f,
                         nullptr),
           RPM_E_INVALID, "gemm M");
    expect(rpm_fno_warm_start(&cfg, (const float*)0x10, &pr, E, 7, (void*)0x10, (void*)0x10, 1, nullptr),
           RPM_E_INVALID, "warm start config");
    std::printf("abi driver done\n");
    return fails ? 1 : 0;
}
