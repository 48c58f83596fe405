// Driver of the library's host code (prime chain, ChaCha20 streams, the
// binary128 slot encoder, the Chebyshev coefficients) under AddressSanitizer
// and UndefinedBehaviorSanitizer (test infrastructure; built and run by
// tests/test_sanitizers.py).  Each call is checked against a property it
// must satisfy, so the run is also a small functional test.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../paper_2412_15126_amd/csrc/host_math.h"

using namespace ckr;

static int fails = 0;
#define CHECK(c, ...)                        \
    do {                                     \
        if (!(c)) {                          \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fputc('\n', stderr);        \
            fails++;                         \
        }                                    \
    } while (0)

int main() {
    // prime chains of a small and a full-size ring: every modulus is prime,
    // 1 mod 2n, distinct, and psi is a primitive 2n-th root of unity
    const int sets[2][7] = {{10, 8, 44, 36, 3, 46, 3}, {16, 24, 50, 40, 7, 50, 3}};
    for (auto &a : sets) {
        Params P = make_params(a[0], a[1], a[2], a[3], a[4], a[5], a[6]);
        CHECK((int)P.mod.size() == P.nmod() && (int)P.psi.size() == P.nmod(), "chain sizes");
        for (int i = 0; i < P.nmod(); i++) {
            u64 q = P.mod[i];
            CHECK(hprime(q) && q % (2 * P.n) == 1, "modulus %d = %llu", i, (unsigned long long)q);
            CHECK(hpow(P.psi[i], P.n, q) == q - 1, "psi^n != -1 for modulus %d", i);
            for (int j = 0; j < i; j++) CHECK(P.mod[j] != q, "repeated modulus %d", i);
            CHECK(hmul(hinv(P.psi[i], q), P.psi[i], q) == 1, "inverse of psi");
        }
        CHECK((int)P.scale.size() == P.nq, "scales");
    }
    bool threw = false;
    try {
        make_params(10, 8, 70, 36, 3, 46, 3);  // q0 beyond the exact-double range
    } catch (const Error &) {
        threw = true;
    }
    CHECK(threw, "an out-of-range prime size must be rejected");

    // ChaCha20 streams: draws stay in range, equal seeds give equal streams
    uint8_t key[32];
    for (int i = 0; i < 32; i++) key[i] = (uint8_t)(7 * i + 1);
    Stream s1(key, kSecret, 3), s2(key, kSecret, 3), s3(key, kPkE, 3);
    int diff = 0;
    for (int i = 0; i < 5000; i++) {
        u64 q = (1ull << 50) - 27;
        u64 u = s1.uniform(q);
        CHECK(u < q, "uniform out of range");
        CHECK(u == s2.uniform(q), "streams of one seed differ");
        int t = s3.ternary(), c = s3.cbd21();
        CHECK(t >= -1 && t <= 1, "ternary %d", t);
        CHECK(c >= -21 && c <= 21, "cbd21 %d", c);
        diff += t != 0;
    }
    CHECK(diff > 2500 && diff < 4000, "ternary density %d of 5000", diff);

    // encoder: decode(encode(z)) = z at the scale's resolution, for a full
    // and a partial slot vector
    for (int logn : {10, 12}) {
        const u32 h = 1u << (logn - 1);
        for (u32 count : {h, 37u}) {
            std::vector<double> z(count), back(count);
            for (u32 k = 0; k < count; k++) z[k] = std::sin(0.37 * k) * 0.9;
            std::vector<i64> m((size_t)1 << logn);
            CHECK(encode_slots(logn, z.data(), count, std::ldexp(1.0, 36), m.data()), "encode");
            decode_slots(logn, m.data(), std::ldexp(1.0, 36), count, back.data());
            double e = 0;
            for (u32 k = 0; k < count; k++) e = std::fmax(e, std::fabs(back[k] - z[k]));
            CHECK(e < 1e-8, "encode/decode error %g at logn %d count %u", e, logn, count);
        }
    }
    {
        std::vector<double> z(4, 1e9);
        std::vector<i64> m(1024);
        CHECK(!encode_slots(10, z.data(), 4, std::ldexp(1.0, 40), m.data()), "overflow must be reported");
    }

    // Chebyshev interpolant of the step: at its nodes it is 1 for d > 0 and 0 for d < 0
    for (int D : {3, 6, 10}) {
        const int M = 1 << (D - 1);
        std::vector<double> c(M);
        cheb_step_coeffs(D, c.data());
        for (int j = 0; j < M; j++) {
            double x = std::cos(M_PI * (j + 0.5) / M), t0 = 1, t1 = x, p = c[0];
            for (int k = 1; k < M; k++) {
                p += c[k] * t1;
                double t2 = 2 * x * t1 - t0;
                t0 = t1;
                t1 = t2;
            }
            CHECK(std::fabs(p - (x > 0 ? 1.0 : 0.0)) < 1e-9, "interpolant at node %d of D=%d: %f", j, D, p);
        }
    }

    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("host driver: all checks passed\n");
    return 0;
}
