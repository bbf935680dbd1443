// Test infrastructure: the host-side validation of libkgs's C ABI under
// AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
// tests/test_sanitizers.py on the CPU).  Every call here is refused or
// answered before the library touches a device, so no GPU is needed; the
// run prints "ok" and returns 0 when every status is the documented one.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <limits>

#include "kgs.h"

static int failures = 0;

static void expect(int got, int want, const char *what)
{
    if (got != want) {
        std::printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want,
                    kgs_last_error(nullptr));
        ++failures;
    }
}

static kgs_config good()
{
    kgs_config c;
    std::memset(&c, 0, sizeof(c));
    c.dim = 2;
    c.n = 8;
    c.lo = -1.0;
    c.hi = 1.0;
    c.tau = 0.01;
    c.kappa1 = c.kappa2 = c.mu = c.gamma = 1.0;
    c.precision = KGS_FP64;
    return c;
}

static int init_status(const kgs_config *c)
{
    double d = 0.0;
    kgs_sim *s = reinterpret_cast<kgs_sim *>(0x1);
    const int rc = kgs_init(c, &d, &d, &d, &d, KGS_HOST, nullptr, &s);
    if (s != nullptr) {
        std::printf("FAIL handle not cleared on error\n");
        ++failures;
    }
    return rc;
}

int main()
{
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    kgs_config c;
    expect(init_status(nullptr), KGS_EINVAL, "null config");
    c = good(); c.dim = 0; expect(init_status(&c), KGS_EINVAL, "dim 0");
    c = good(); c.dim = 4; expect(init_status(&c), KGS_EINVAL, "dim 4");
    c = good(); c.n = 0; expect(init_status(&c), KGS_EINVAL, "n 0");
    c = good(); c.n = 7; expect(init_status(&c), KGS_EODDN, "odd n");
    c = good(); c.hi = -1.0; expect(init_status(&c), KGS_EINVAL, "empty box");
    c = good(); c.hi = inf; expect(init_status(&c), KGS_EINVAL, "infinite box");
    c = good(); c.tau = 0.0; expect(init_status(&c), KGS_EINVAL, "tau 0");
    c = good(); c.tau = nan; expect(init_status(&c), KGS_EINVAL, "tau NaN");
    c = good(); c.kappa1 = nan; expect(init_status(&c), KGS_EINVAL, "kappa1 NaN");
    c = good(); c.gamma = inf; expect(init_status(&c), KGS_EINVAL, "gamma inf");
    c = good(); c.precision = 2; expect(init_status(&c), KGS_EINVAL, "precision 2");
    c = good(); c.reserved = 1; expect(init_status(&c), KGS_EINVAL, "reserved");
    c = good(); c.n = 1 << 20; c.dim = 3; expect(init_status(&c), KGS_EINVAL, "too large");
    // det = 1 + beta tau'/2 = 0 with tau' = 0.5, h = 0.25, mu = 0, kappa2 = -0.5
    c = good(); c.dim = 1; c.tau = 1.0; c.kappa2 = -0.5; c.mu = 0.0;
    expect(init_status(&c), KGS_ESINGULAR, "singular (u, v) matrix");
    double d = 0.0;
    kgs_sim *s = nullptr;
    c = good();
    expect(kgs_init(&c, nullptr, &d, &d, &d, KGS_HOST, nullptr, &s), KGS_EINVAL, "null field");
    expect(kgs_init(&c, &d, &d, &d, &d, 7, nullptr, &s), KGS_EINVAL, "bad memory kind");
    expect(kgs_init(&c, &d, &d, &d, &d, KGS_HOST, nullptr, nullptr), KGS_EINVAL, "null out");
    expect(kgs_step(nullptr, 1), KGS_EINVAL, "step on null");
    expect(kgs_energy(nullptr, &d), KGS_EINVAL, "energy on null");
    expect(kgs_sync(nullptr), KGS_EINVAL, "sync on null");
    expect(kgs_free(nullptr), KGS_OK, "free null");
    // required bytes: two states for ping-pong kernels, one otherwise, 0 if invalid
    for (int dim = 1; dim <= 3; ++dim)
        for (int n : {2, 64, 130, 256})
            for (int prec : {KGS_FP64, KGS_FP32}) {
                c = good();
                c.dim = dim;
                c.n = n;
                c.precision = prec;
                const double pts = std::pow(static_cast<double>(n), dim);
                const double state = 4.0 * pts * (prec == KGS_FP64 ? 8 : 4);
                const double got = static_cast<double>(kgs_required_bytes(&c));
                if (!(got >= state && got < 2.0 * state + (1 << 21))) {
                    std::printf("FAIL required bytes dim=%d n=%d prec=%d: %.0f\n", dim, n, prec, got);
                    ++failures;
                }
            }
    c = good(); c.n = 9;
    if (kgs_required_bytes(&c) != 0) { std::printf("FAIL required bytes of odd n\n"); ++failures; }
    // kgs_step_fields: every refusal comes before the device
    c = good();
    double *p = &d;
    expect(kgs_step_fields(nullptr, p, p, p, p, 1, nullptr), KGS_EINVAL, "fields: null config");
    expect(kgs_step_fields(&c, nullptr, p, p, p, 1, nullptr), KGS_EINVAL, "fields: null array");
    expect(kgs_step_fields(&c, p, p, p, p, -1, nullptr), KGS_EINVAL, "fields: negative steps");
    c.dim = 3; c.n = 130;
    expect(kgs_step_fields(&c, p, p, p, p, 1, nullptr), KGS_ENOMEM, "fields: beyond scratch");
    for (int st = -1; st <= 7; ++st)
        if (kgs_status_string(st) == nullptr) { std::printf("FAIL status string\n"); ++failures; }
    if (kgs_last_error(nullptr) == nullptr) { std::printf("FAIL last error\n"); ++failures; }
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
