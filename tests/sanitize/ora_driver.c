/* Driver of the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (test infrastructure; built and run by tests/test_sanitizers.py).
 *
 * The oracle's source is compiled into this one translation unit so that
 * every function, static helpers included, is instrumented.  The driver runs
 * each circuit family once on a small ring (n = 2^10, 8 values) and checks
 * the decoded results against the plaintext answer, so a sanitizer report
 * comes with a run that still computes the right thing.  Every object is
 * freed, so LeakSanitizer sees the whole lifetime. */
#include "../../oracle/ora.c"

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { fprintf(stderr, __VA_ARGS__); fputc('\n', stderr); fails++; } } while (0)

/* 8 values with gap >= 0.05 in [0, 1), and their 1-based ranks */
static const double V8[8] = {0.61, 0.05, 0.83, 0.27, 0.44, 0.97, 0.16, 0.72};
static const int R8[8] = {5, 1, 7, 3, 4, 8, 2, 6};

static void check_ranks(const ora_keys *K, const ora_ct *c, const char *what) {
    double z[8];
    ora_decrypt(K, c, z, 8);
    for (int i = 0; i < 8; i++)
        CHECK(fabs(z[i] - R8[i]) < 0.45, "%s: slot %d = %f, want %d", what, i, z[i], R8[i]);
}

int main(void) {
    ora_set_threads(2);
    /* logn, L, q0_bits, log_scale, K, p_bits, dnum */
    ora_params *P = ora_params_new(10, 36, 44, 36, 9, 40, 4);
    CHECK(P != NULL, "params");
    u32 gal[256];
    int ng = ora_circuit_galois(P, 8, 7, gal); /* rank, order statistics and sort */
    CHECK(ng > 0 && ng <= 256, "galois count %d", ng);
    u8 kseed[32], eseed[32];
    for (int i = 0; i < 32; i++) { kseed[i] = (u8)(i + 1); eseed[i] = (u8)(3 * i + 7); }
    ora_keys *K = ora_keygen(P, kseed, 36, gal, ng);
    int st = 0;

    /* rank with the f/g composite g^2 f, the minimax composite and the Chebyshev comparator */
    const ora_cmp fg = {2, 1, 0, 0}, mm = {0, 0, 0, 4}, ch = {0, 0, 7, 0}, ind = {3, 2, 0, 0};
    const ora_cmp cmps[3] = {fg, mm, ch};
    const char *names[3] = {"rank g^2 f", "rank minimax", "rank chebyshev"};
    for (int t = 0; t < 3; t++) {
        int lvl = ora_rank_depth(cmps[t]);
        ora_ct *v = ora_encrypt(K, V8, 8, lvl, eseed, &st);
        CHECK(v && st == 0, "encrypt %d", st);
        ora_ct *r = ora_rank(K, v, 8, cmps[t], &st);
        CHECK(r && st == 0, "%s status %d", names[t], st);
        if (r) check_ranks(K, r, names[t]);
        ora_ct_free(r);
        ora_ct_free(v);
    }

    /* tie-corrected rank and order statistic k = 3 (value 0.27) */
    {
        int lvl = ora_order_stat_depth(8, 3, fg, ind, 1);
        ora_ct *v = ora_encrypt(K, V8, 8, lvl, eseed, &st);
        ora_ct *oh = NULL, *val = NULL;
        st = ora_order_stat(K, v, 8, 3, fg, ind, 1, &oh, &val);
        CHECK(st == 0, "order statistic status %d", st);
        if (st == 0) {
            double z[8], w;
            ora_decrypt(K, oh, z, 8);
            for (int i = 0; i < 8; i++)
                CHECK(fabs(z[i] - (R8[i] == 3)) < 0.1, "one-hot slot %d = %f", i, z[i]);
            ora_decrypt(K, val, &w, 1);
            CHECK(fabs(w - 0.27) < 0.02, "order statistic value %f", w);
        }
        ora_ct_free(oh);
        ora_ct_free(val);
        ora_ct_free(v);
    }

    /* sort (row form) */
    {
        int lvl = ora_sort_depth(fg, ind);
        CHECK(lvl <= 36, "sort depth %d", lvl);
        ora_ct *v = ora_encrypt(K, V8, 8, lvl, eseed, &st);
        ora_ct *s = ora_sort(K, v, 8, fg, ind, &st);
        CHECK(s && st == 0, "sort status %d", st);
        if (s) {
            double z[8], want[8];
            memcpy(want, V8, sizeof want);
            for (int i = 0; i < 8; i++)
                for (int j = i + 1; j < 8; j++)
                    if (want[j] < want[i]) { double x = want[i]; want[i] = want[j]; want[j] = x; }
            ora_decrypt(K, s, z, 8);
            for (int i = 0; i < 8; i++) CHECK(fabs(z[i] - want[i]) < 0.02, "sorted slot %d = %f", i, z[i]);
        }
        ora_ct_free(s);
        ora_ct_free(v);
    }

    /* multi-ciphertext rank: 2 blocks of 4 (Equation (3)) */
    ora_keys *K4 = NULL;
    {
        u32 g4[256];
        int n4 = ora_circuit_galois(P, 4, 4, g4);
        K4 = ora_keygen(P, kseed, 20, g4, n4);
        int lvl = ora_rank_multi_depth(fg);
        ora_ct *blk[2], *R[2] = {NULL, NULL};
        u8 e2[32];
        memcpy(e2, eseed, 32);
        for (int b = 0; b < 2; b++) {
            e2[0] = (u8)(eseed[0] + b);
            blk[b] = ora_encrypt(K4, V8 + 4 * b, 4, lvl, e2, &st);
        }
        st = ora_rank_multi(K4, blk, 2, 4, fg, R);
        CHECK(st == 0, "multi rank status %d", st);
        if (st == 0)
            for (int b = 0; b < 2; b++) {
                double z[4];
                ora_decrypt(K4, R[b], z, 4);
                for (int i = 0; i < 4; i++)
                    CHECK(fabs(z[i] - R8[4 * b + i]) < 0.45, "block %d slot %d = %f", b, i, z[i]);
            }
        for (int b = 0; b < 2; b++) { ora_ct_free(R[b]); ora_ct_free(blk[b]); }
    }

    /* error paths: too few levels, bad N, missing rotation keys */
    {
        ora_ct *v = ora_encrypt(K, V8, 8, 3, eseed, &st);
        ora_ct *r = ora_rank(K, v, 8, fg, &st);
        CHECK(r == NULL && st == ORA_E_DEPTH, "shallow rank status %d", st);
        r = ora_rank(K, v, 1, fg, &st);
        CHECK(r == NULL && st != 0, "rank of N=1 status %d", st);
        ora_ct_free(v);
        v = ora_encrypt(K4, V8, 8, 20, eseed, &st);
        ora_ct *oh = NULL, *val = NULL;
        st = ora_order_stat(K4, v, 8, 2, fg, ind, 0, &oh, &val);
        CHECK(st == ORA_E_INVALID && !oh && !val, "order statistic without its keys: status %d", st);
        r = ora_sort(K4, v, 8, fg, ind, &st);
        CHECK(r == NULL && st == ORA_E_INVALID, "sort without its keys: status %d", st);
        ora_ct_free(v);
    }

    ora_keys_free(K4);
    ora_keys_free(K);
    ora_params_free(P);
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("oracle driver: all checks passed\n");
    return 0;
}
