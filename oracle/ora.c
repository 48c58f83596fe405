/*
 * ora.c -- CPU oracle for the RNS-CKKS ranking / order-statistics / sorting
 * path (arXiv 2412.15126).  TEST INFRASTRUCTURE ONLY: the product library
 * never includes, links or calls this file; only tests/, the smoke check and
 * the cpu_baseline leg of bench.py do.
 *
 * Plain and slow on purpose.  Every residue is a canonical uint64 in [0, q);
 * products are reduced with unsigned __int128 '%'.  Polynomials are held in
 * the coefficient domain; a ring product is "transform both, multiply
 * pointwise, transform back" with a textbook radix-2 NTT.  Nothing is fused
 * or reordered beyond the definitions below.
 *
 * What the paper fixes (section 2.1 "CKKS Scheme"): ring Z_q[x]/(x^n+1),
 * n/2 complex slots, ct+ct, ct*ct, left/right slot rotations, ct-pt ops.
 * Everything underneath is the standard full-RNS CKKS construction (CKKS
 * 2017; full-RNS variant with fast base conversion; hybrid key switching
 * with dnum digits), which the paper uses through OpenFHE.  The readings
 * taken where the paper is silent are:
 *   - primes:   special primes = largest primes < 2^p_bits, q_0 = largest
 *               unused prime < 2^q0_bits, rescale primes q_L..q_1 chosen
 *               greedily as the unused prime nearest the running scale;
 *               every prime is 1 mod 2n.
 *   - scales:   D_L = 2^log_scale, D_{l-1} = (D_l * D_l) / q_l (double);
 *               every ciphertext at level l carries scale D_l.
 *   - sampling: ChaCha20 (RFC 8439) keyed by a 32-byte seed, nonce =
 *               (purpose, object id); ternary secret by 2-bit rejection,
 *               errors centred binomial eta=21, uniform residues by
 *               bit-mask rejection; all samples in the coefficient domain.
 *   - encoding: slot k <-> root zeta^(5^k mod 2n), zeta = exp(i*pi/n);
 *               m_j = round_half_away((2*D/n) * Re DFT_2n(w)[j]) with w the
 *               slot vector scattered to positions 5^k mod 2n; evaluated in
 *               binary128 so the rounding is that of the exact value.
 *   - key switching: fast base conversion without correction in ModUp;
 *               ModDown and rescale round (X + (m - 1)/2 before the floor
 *               division by m, m = P or q_l): rescale is (c_i - [v]_{q_i}) *
 *               q_l^{-1} with v the last limb's residue in (-q_l/2, q_l/2);
 *               ModDown's conversion removes its overflow u = floor(sum_i
 *               y_i / p_i) (evaluated in IEEE double, in source order), so
 *               ModDown is round(X / P).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#include <math.h>
#include <quadmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;
typedef uint8_t u8;
typedef unsigned __int128 u128;

#define ORA_MAXMOD 128

/* status codes (same meaning as the product's) */
#define ORA_OK 0
#define ORA_E_INVALID (-1)
#define ORA_E_RANGE (-2)
#define ORA_E_DEPTH (-3)

/* comparator: the f/g composite of section 2.2, g applied dg times then f
 * applied df times; or the Chebyshev interpolant of Eq. (1) with cheb levels;
 * or the first mm stages of the minimax composite (the other fields 0) */
typedef struct { int dg, df, cheb, mm; } ora_cmp;

/* ------------------------------------------------------------------ */
/* modular arithmetic on canonical residues                            */
/* ------------------------------------------------------------------ */
static u64 mulm(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addm(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }
static u64 powm(u64 a, u64 e, u64 q) {
    u64 r = 1 % q; a %= q;
    while (e) { if (e & 1) r = mulm(r, a, q); a = mulm(a, a, q); e >>= 1; }
    return r;
}
static u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); } /* q prime */
static u64 red_i64(i64 v, u64 q) {
    i64 r = v % (i64)q;
    if (r < 0) r += (i64)q;
    return (u64)r;
}

/* Miller-Rabin with the first twelve prime bases: deterministic below 2^64 */
static int is_prime(u64 n) {
    static const u64 B[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) if (n % B[i] == 0) return n == B[i];
    u64 d = n - 1; int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powm(B[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) {
            x = mulm(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* parameters                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    int logn; u64 n;
    int L;        /* top level; the q chain is q_0..q_L */
    int nq;       /* L + 1 */
    int K;        /* special primes */
    int dnum, alpha;
    int log_scale;
    u64 mod[ORA_MAXMOD];      /* [0, nq): q chain, [nq, nq+K): special primes */
    u64 psi[ORA_MAXMOD];      /* primitive 2n-th root of unity per modulus */
    double scale[ORA_MAXMOD]; /* D_l for l = 0..L */
} ora_params;

static int in_list(u64 c, const u64 *list, int cnt) {
    for (int i = 0; i < cnt; i++) if (list[i] == c) return 1;
    return 0;
}

static u64 largest_below(int bits, u64 m, const u64 *ex, int nex) {
    u64 top = (bits >= 64) ? ~0ULL : ((1ULL << bits) - 1);
    u64 c = top - ((top - 1) % m); /* largest value <= top that is 1 mod m */
    for (; c > m; c -= m)
        if (!in_list(c, ex, nex) && is_prime(c)) return c;
    return 0;
}

/* unused prime = 1 mod m nearest to T; equal distance prefers the smaller */
static u64 nearest_to(double T, u64 m, const u64 *ex, int nex) {
    u64 f = (u64)floor(T);
    u64 lo = f - ((f - 1) % m);
    u64 hi = lo + m;
    for (;;) {
        double dlo = T - (double)lo, dhi = (double)hi - T;
        if (dlo <= dhi) {
            if (!in_list(lo, ex, nex) && is_prime(lo)) return lo;
            lo -= m;
        } else {
            if (!in_list(hi, ex, nex) && is_prime(hi)) return hi;
            hi += m;
        }
    }
}

static u64 find_psi(u64 q, u64 n) {
    for (u64 x = 2;; x++) {
        u64 w = powm(x, (q - 1) / (2 * n), q);
        if (powm(w, n, q) == q - 1) return w;
    }
}

ora_params *ora_params_new(int logn, int L, int q0_bits, int log_scale, int K, int p_bits, int dnum) {
    if (logn < 2 || logn > 17 || L < 0 || L + 1 + K > ORA_MAXMOD || dnum < 1 || dnum > L + 1) return NULL;
    if (q0_bits > 50 || p_bits > 50 || log_scale > 48) return NULL;
    ora_params *P = (ora_params *)calloc(1, sizeof(ora_params));
    P->logn = logn; P->n = 1ULL << logn; P->L = L; P->nq = L + 1; P->K = K;
    P->dnum = dnum; P->alpha = (L + 1 + dnum - 1) / dnum; P->log_scale = log_scale;
    u64 m = 2 * P->n;
    u64 used[ORA_MAXMOD]; int nu = 0;
    for (int k = 0; k < K; k++) { u64 p = largest_below(p_bits, m, used, nu); used[nu++] = p; P->mod[P->nq + k] = p; }
    P->mod[0] = largest_below(q0_bits, m, used, nu); used[nu++] = P->mod[0];
    double D = ldexp(1.0, log_scale);
    P->scale[L] = D;
    for (int l = L; l >= 1; l--) {
        u64 q = nearest_to(P->scale[l], m, used, nu);
        used[nu++] = q; P->mod[l] = q;
        P->scale[l - 1] = (P->scale[l] * P->scale[l]) / (double)q;
    }
    for (int t = 0; t < P->nq + K; t++) P->psi[t] = find_psi(P->mod[t], P->n);
    return P;
}
void ora_params_free(ora_params *P) { free(P); }

/* mods: nq+K values, scales: nq values, psi: nq+K values */
void ora_params_info(const ora_params *P, u64 *mods, double *scales, u64 *psi, int *dims) {
    for (int t = 0; t < P->nq + P->K; t++) { if (mods) mods[t] = P->mod[t]; if (psi) psi[t] = P->psi[t]; }
    for (int l = 0; l < P->nq; l++) if (scales) scales[l] = P->scale[l];
    if (dims) { dims[0] = P->logn; dims[1] = P->L; dims[2] = P->K; dims[3] = P->dnum; dims[4] = P->alpha; }
}

static int g_threads = 1;
void ora_set_threads(int t) {
    g_threads = t < 1 ? 1 : t;
#ifdef _OPENMP
    omp_set_num_threads(g_threads);
#endif
}

/* ------------------------------------------------------------------ */
/* textbook NTT: cyclic radix-2 Cooley-Tukey with bit reversal, plus   */
/* the x^n+1 twist (a_j * psi^j) so that output k = a(psi^(2k+1)).     */
/* ------------------------------------------------------------------ */
static void bitrev_permute(u64 *a, u64 n) {
    for (u64 i = 1, j = 0; i < n; i++) {
        u64 bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}

static void ntt_cyclic(u64 *a, u64 n, u64 q, u64 w) {
    bitrev_permute(a, n);
    for (u64 len = 2; len <= n; len <<= 1) {
        u64 wl = powm(w, n / len, q);
        for (u64 i = 0; i < n; i += len) {
            u64 wj = 1;
            for (u64 j = 0; j < len / 2; j++) {
                u64 u = a[i + j], v = mulm(a[i + j + len / 2], wj, q);
                a[i + j] = addm(u, v, q);
                a[i + j + len / 2] = subm(u, v, q);
                wj = mulm(wj, wl, q);
            }
        }
    }
}

static void ntt_fwd(u64 *a, u64 n, u64 q, u64 psi) {
    u64 pj = 1;
    for (u64 j = 0; j < n; j++) { a[j] = mulm(a[j], pj, q); pj = mulm(pj, psi, q); }
    ntt_cyclic(a, n, q, mulm(psi, psi, q));
}

static void ntt_inv(u64 *a, u64 n, u64 q, u64 psi) {
    u64 ipsi = invm(psi, q);
    ntt_cyclic(a, n, q, mulm(ipsi, ipsi, q));
    u64 ninv = invm(n % q, q), pj = ninv;
    for (u64 j = 0; j < n; j++) { a[j] = mulm(a[j], pj, q); pj = mulm(pj, ipsi, q); }
}

/* pin helper: c = a*b mod (x^n+1, q) */
void ora_negacyclic_mul(u64 n, u64 q, u64 psi, const u64 *a, const u64 *b, u64 *c) {
    u64 *A = (u64 *)malloc(n * 8), *B = (u64 *)malloc(n * 8);
    memcpy(A, a, n * 8); memcpy(B, b, n * 8);
    ntt_fwd(A, n, q, psi); ntt_fwd(B, n, q, psi);
    for (u64 i = 0; i < n; i++) c[i] = mulm(A[i], B[i], q);
    ntt_inv(c, n, q, psi);
    free(A); free(B);
}
/* pin helper: forward transform only (output k = a(psi^(2k+1))) */
void ora_ntt_forward(u64 n, u64 q, u64 psi, u64 *a) { ntt_fwd(a, n, q, psi); }

/* ------------------------------------------------------------------ */
/* ChaCha20 block function (RFC 8439 section 2.3) and samplers         */
/* ------------------------------------------------------------------ */
static u32 rotl32(u32 x, int k) { return (x << k) | (x >> (32 - k)); }
#define QR(a, b, c, d) \
    a += b; d ^= a; d = rotl32(d, 16); c += d; b ^= c; b = rotl32(b, 12); \
    a += b; d ^= a; d = rotl32(d, 8);  c += d; b ^= c; b = rotl32(b, 7);

static u32 ld32(const u8 *p) { return (u32)p[0] | ((u32)p[1] << 8) | ((u32)p[2] << 16) | ((u32)p[3] << 24); }

void ora_chacha20_block(const u8 key[32], u32 counter, const u8 nonce[12], u32 out[16]) {
    u32 s[16];
    s[0] = 0x61707865; s[1] = 0x3320646e; s[2] = 0x79622d32; s[3] = 0x6b206574;
    for (int i = 0; i < 8; i++) s[4 + i] = ld32(key + 4 * i);
    s[12] = counter;
    for (int i = 0; i < 3; i++) s[13 + i] = ld32(nonce + 4 * i);
    u32 x[16];
    memcpy(x, s, sizeof s);
    for (int r = 0; r < 10; r++) {
        QR(x[0], x[4], x[8], x[12]); QR(x[1], x[5], x[9], x[13]);
        QR(x[2], x[6], x[10], x[14]); QR(x[3], x[7], x[11], x[15]);
        QR(x[0], x[5], x[10], x[15]); QR(x[1], x[6], x[11], x[12]);
        QR(x[2], x[7], x[8], x[13]); QR(x[3], x[4], x[9], x[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = x[i] + s[i];
}

typedef struct { u8 key[32]; u8 nonce[12]; u32 counter; u32 buf[16]; int pos; } stream_t;

static void stream_init(stream_t *st, const u8 key[32], u32 purpose, u64 id) {
    memcpy(st->key, key, 32);
    for (int i = 0; i < 4; i++) st->nonce[i] = (u8)(purpose >> (8 * i));
    for (int i = 0; i < 8; i++) st->nonce[4 + i] = (u8)(id >> (8 * i));
    st->counter = 0; st->pos = 16;
}
static u32 next32(stream_t *st) {
    if (st->pos == 16) { ora_chacha20_block(st->key, st->counter++, st->nonce, st->buf); st->pos = 0; }
    return st->buf[st->pos++];
}
static u64 next64(stream_t *st) { u64 lo = next32(st); u64 hi = next32(st); return lo | (hi << 32); }

static int samp_ternary(stream_t *st) {
    for (;;) { u32 v = next32(st) & 3u; if (v != 3u) return (int)v - 1; }
}
static int samp_cbd21(stream_t *st) {
    u64 w = next64(st);
    return __builtin_popcountll(w & 0x1FFFFFULL) - __builtin_popcountll((w >> 21) & 0x1FFFFFULL);
}
static u64 samp_uniform(stream_t *st, u64 q) {
    int bits = 64 - __builtin_clzll(q);
    u64 mask = (bits == 64) ? ~0ULL : ((1ULL << bits) - 1);
    for (;;) { u64 w = next64(st) & mask; if (w < q) return w; }
}

enum { PUR_SECRET = 1, PUR_PK_A = 2, PUR_PK_E = 3, PUR_KS_A = 4, PUR_KS_E = 5,
       PUR_ENC_U = 6, PUR_ENC_E0 = 7, PUR_ENC_E1 = 8 };

/* pin helper: kind 0 ternary, 1 cbd21, 2 uniform mod q */
void ora_sample(const u8 key[32], u32 purpose, u64 id, int kind, u64 q, u64 count, i64 *out) {
    stream_t st; stream_init(&st, key, purpose, id);
    for (u64 i = 0; i < count; i++)
        out[i] = kind == 0 ? samp_ternary(&st) : kind == 1 ? samp_cbd21(&st) : (i64)samp_uniform(&st, q);
}

/* ------------------------------------------------------------------ */
/* encoding / decoding                                                 */
/* ------------------------------------------------------------------ */
static u64 slot_root_exp(u64 k, u64 n) { return powm(5, k, 2 * n); } /* 5^k mod 2n */

static __float128 round_half_away(__float128 x) {
    return x >= 0 ? floorq(x + 0.5Q) : -floorq(-x + 0.5Q);
}

/* textbook radix-2 complex DFT in binary128: F[j] = sum_t x[t] exp(-2 pi i j t / M) */
static void fft_q(__complex128 *x, u64 M) {
    for (u64 i = 1, j = 0; i < M; i++) {
        u64 bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { __complex128 t = x[i]; x[i] = x[j]; x[j] = t; }
    }
    __complex128 *tw = (__complex128 *)malloc(sizeof(__complex128) * (M / 2));
    for (u64 k = 0; k < M / 2; k++) {
        __float128 ang = -2.0Q * M_PIq * (__float128)k / (__float128)M;
        __real__ tw[k] = cosq(ang); __imag__ tw[k] = sinq(ang);
    }
    for (u64 len = 2; len <= M; len <<= 1) {
        u64 step = M / len;
        for (u64 i = 0; i < M; i += len)
            for (u64 j = 0; j < len / 2; j++) {
                __complex128 u = x[i + j], v = x[i + j + len / 2] * tw[j * step];
                x[i + j] = u + v; x[i + j + len / 2] = u - v;
            }
    }
    free(tw);
}

/* z: real slot values for slots [0, count); others zero.  m: n signed ints. */
int ora_encode(const ora_params *P, const double *z, u32 count, double scale, i64 *m) {
    u64 n = P->n, M = 2 * n;
    if (count > n / 2) return ORA_E_RANGE;
    __complex128 *w = (__complex128 *)calloc(M, sizeof(__complex128));
    for (u64 k = 0; k < count; k++) __real__ w[slot_root_exp(k, n)] = (__float128)z[k];
    fft_q(w, M);
    __float128 f = 2.0Q * (__float128)scale / (__float128)n;
    int st = ORA_OK;
    for (u64 j = 0; j < n; j++) {
        __float128 r = round_half_away(f * crealq(w[j]));
        if (fabsq(r) > 0x1p62Q) { st = ORA_E_RANGE; r = 0; }
        m[j] = (i64)r;
    }
    free(w);
    return st;
}

/* real parts of slots [0, count) of m / scale */
void ora_decode(const ora_params *P, const i64 *m, double scale, u32 count, double *z) {
    u64 n = P->n, M = 2 * n;
    long double *ct = (long double *)malloc(sizeof(long double) * M);
    for (u64 t = 0; t < M; t++) ct[t] = cosl(2.0L * 3.14159265358979323846264338327950288L * (long double)t / (long double)M);
    for (u32 k = 0; k < count; k++) {
        u64 g = slot_root_exp(k, n);
        long double acc = 0;
        for (u64 j = 0; j < n; j++) acc += (long double)m[j] * ct[(j * g) % M];
        z[k] = (double)(acc / (long double)scale);
    }
    free(ct);
}

/* ------------------------------------------------------------------ */
/* RNS polynomials, ciphertexts and keys                               */
/* ------------------------------------------------------------------ */
typedef struct { const ora_params *P; int level; u64 *d; } ora_ct; /* d: [2][level+1][n], coefficient domain */

typedef struct { u32 g; u64 *d; } ora_swk; /* d: [beta_max][2][lmax+1+K][n], NTT form */

typedef struct {
    const ora_params *P;
    int lmax;
    i64 *s;         /* ternary secret, n values */
    u64 *pk;        /* [2][lmax+1][n] coefficient domain */
    int nswk;
    ora_swk *swk;   /* index 0 = relinearisation key (g = 0) */
} ora_keys;

#define LIMB(base, t, n) ((base) + (size_t)(t) * (n))

static ora_ct *ct_new(const ora_params *P, int level) {
    ora_ct *c = (ora_ct *)malloc(sizeof(ora_ct));
    c->P = P; c->level = level;
    c->d = (u64 *)calloc((size_t)2 * (level + 1) * P->n, 8);
    return c;
}
static u64 *ct_poly(const ora_ct *c, int p) { return c->d + (size_t)p * (c->level + 1) * c->P->n; }
static ora_ct *ct_copy(const ora_ct *a) {
    ora_ct *c = ct_new(a->P, a->level);
    memcpy(c->d, a->d, (size_t)2 * (a->level + 1) * a->P->n * 8);
    return c;
}
void ora_ct_free(ora_ct *c) { if (c) { free(c->d); free(c); } }
int ora_ct_level(const ora_ct *c) { return c->level; }
double ora_ct_scale(const ora_ct *c) { return c->P->scale[c->level]; }
void ora_ct_export(const ora_ct *c, u64 *out) { memcpy(out, c->d, (size_t)2 * (c->level + 1) * c->P->n * 8); }
ora_ct *ora_ct_import(const ora_params *P, int level, const u64 *data) {
    ora_ct *c = ct_new(P, level);
    memcpy(c->d, data, (size_t)2 * (level + 1) * P->n * 8);
    return c;
}

/* c = a * b for one limb, all in coefficient domain */
static void ring_mul_limb(const u64 *a, const u64 *b, u64 *c, const ora_params *P, int t) {
    u64 n = P->n, q = P->mod[t];
    u64 *A = (u64 *)malloc(n * 8), *B = (u64 *)malloc(n * 8);
    memcpy(A, a, n * 8); memcpy(B, b, n * 8);
    ntt_fwd(A, n, q, P->psi[t]); ntt_fwd(B, n, q, P->psi[t]);
    for (u64 i = 0; i < n; i++) c[i] = mulm(A[i], B[i], q);
    ntt_inv(c, n, q, P->psi[t]);
    free(A); free(B);
}

/* sigma_g on one limb in the coefficient domain: x^j -> x^(j*g mod 2n), x^n = -1 */
static void automorph_limb(const u64 *a, u64 *b, u64 n, u64 q, u64 g) {
    for (u64 j = 0; j < n; j++) {
        u64 e = (j * g) % (2 * n);
        if (e < n) b[e] = a[j];
        else b[e - n] = a[j] ? q - a[j] : 0;
    }
}
void ora_automorphism(u64 n, u64 q, u64 g, const u64 *a, u64 *b) { automorph_limb(a, b, n, q, g); }

/* index of the key limb that holds modulus index mt (q_0..q_lmax, then p_0..) */
static int key_limb(const ora_params *P, int lmax, int mt) { return mt < P->nq ? mt : lmax + 1 + (mt - P->nq); }

static void gen_swk(ora_keys *Kp, ora_swk *w, const u64 *s_prime_coeff /* [nq+K][n] residues of s' */,
                    const u8 seed[32]) {
    const ora_params *P = Kp->P;
    u64 n = P->n; int lmax = Kp->lmax, E = lmax + 1 + P->K;
    int beta = (lmax + 1 + P->alpha - 1) / P->alpha;
    w->d = (u64 *)calloc((size_t)beta * 2 * E * n, 8);
    u64 Pmod[ORA_MAXMOD];
    for (int t = 0; t < P->nq; t++) {
        u64 q = P->mod[t], acc = 1 % q;
        for (int k = 0; k < P->K; k++) acc = mulm(acc, P->mod[P->nq + k] % q, q);
        Pmod[t] = acc;
    }
    for (int j = 0; j < beta; j++) {
        i64 *e = (i64 *)malloc(n * sizeof(i64));
        stream_t st; stream_init(&st, seed, PUR_KS_E, ((u64)w->g << 32) | ((u64)j << 16));
        for (u64 i = 0; i < n; i++) e[i] = samp_cbd21(&st);
        #pragma omp parallel for schedule(dynamic)
        for (int li = 0; li < E; li++) {
            int mt = li <= lmax ? li : P->nq + (li - lmax - 1);
            u64 q = P->mod[mt];
            u64 *a = (u64 *)malloc(n * 8), *sa = (u64 *)malloc(n * 8), *sl = (u64 *)malloc(n * 8);
            stream_t sta; stream_init(&sta, seed, PUR_KS_A, ((u64)w->g << 32) | ((u64)j << 16) | (u64)mt);
            for (u64 i = 0; i < n; i++) a[i] = samp_uniform(&sta, q);
            for (u64 i = 0; i < n; i++) sl[i] = red_i64(Kp->s[i], q);
            ring_mul_limb(a, sl, sa, P, mt); /* a*s */
            u64 *b = LIMB(w->d, ((size_t)j * 2 + 0) * E + li, n);
            u64 *A = LIMB(w->d, ((size_t)j * 2 + 1) * E + li, n);
            int in_digit = mt < P->nq && mt >= j * P->alpha && mt < (j + 1) * P->alpha;
            for (u64 i = 0; i < n; i++) {
                u64 v = subm(red_i64(e[i], q), sa[i], q);
                if (in_digit) v = addm(v, mulm(Pmod[mt], LIMB(s_prime_coeff, mt, n)[i], q), q);
                b[i] = v;
            }
            memcpy(A, a, n * 8);
            ntt_fwd(b, n, q, P->psi[mt]);
            ntt_fwd(A, n, q, P->psi[mt]);
            free(a); free(sa); free(sl);
        }
        free(e);
    }
}

/* gal: Galois elements of the rotation keys wanted (the relinearisation key is always made) */
ora_keys *ora_keygen(const ora_params *P, const u8 seed[32], int lmax, const u32 *gal, int ngal) {
    if (lmax < 0 || lmax > P->L) return NULL;
    u64 n = P->n;
    ora_keys *Kp = (ora_keys *)calloc(1, sizeof(ora_keys));
    Kp->P = P; Kp->lmax = lmax;
    Kp->s = (i64 *)malloc(n * sizeof(i64));
    { stream_t st; stream_init(&st, seed, PUR_SECRET, 0); for (u64 i = 0; i < n; i++) Kp->s[i] = samp_ternary(&st); }
    /* public key */
    Kp->pk = (u64 *)calloc((size_t)2 * (lmax + 1) * n, 8);
    {
        i64 *e = (i64 *)malloc(n * sizeof(i64));
        stream_t st; stream_init(&st, seed, PUR_PK_E, 0);
        for (u64 i = 0; i < n; i++) e[i] = samp_cbd21(&st);
        #pragma omp parallel for schedule(dynamic)
        for (int t = 0; t <= lmax; t++) {
            u64 q = P->mod[t];
            u64 *a = LIMB(Kp->pk, (lmax + 1) + t, n), *b = LIMB(Kp->pk, t, n);
            u64 *sl = (u64 *)malloc(n * 8), *sa = (u64 *)malloc(n * 8);
            stream_t sta; stream_init(&sta, seed, PUR_PK_A, (u64)t);
            for (u64 i = 0; i < n; i++) a[i] = samp_uniform(&sta, q);
            for (u64 i = 0; i < n; i++) sl[i] = red_i64(Kp->s[i], q);
            ring_mul_limb(a, sl, sa, P, t);
            for (u64 i = 0; i < n; i++) b[i] = subm(red_i64(e[i], q), sa[i], q);
            free(sl); free(sa);
        }
        free(e);
    }
    /* switching keys: index 0 relinearisation (s' = s^2), then rotations (s' = sigma_g(s)) */
    int nm = P->nq + P->K;
    Kp->nswk = 1 + ngal;
    Kp->swk = (ora_swk *)calloc(Kp->nswk, sizeof(ora_swk));
    u64 *sp = (u64 *)calloc((size_t)nm * n, 8);
    for (int w = 0; w < Kp->nswk; w++) {
        u32 g = w == 0 ? 0u : gal[w - 1];
        Kp->swk[w].g = g;
        #pragma omp parallel for schedule(dynamic)
        for (int mt = 0; mt < nm; mt++) {
            int live = mt <= lmax || mt >= P->nq;
            if (!live) continue;
            u64 q = P->mod[mt];
            u64 *sl = (u64 *)malloc(n * 8);
            for (u64 i = 0; i < n; i++) sl[i] = red_i64(Kp->s[i], q);
            if (g == 0) ring_mul_limb(sl, sl, LIMB(sp, mt, n), P, mt);
            else automorph_limb(sl, LIMB(sp, mt, n), n, q, g);
            free(sl);
        }
        gen_swk(Kp, &Kp->swk[w], sp, seed);
    }
    free(sp);
    return Kp;
}

void ora_keys_free(ora_keys *Kp) {
    if (!Kp) return;
    for (int w = 0; w < Kp->nswk; w++) free(Kp->swk[w].d);
    free(Kp->swk); free(Kp->s); free(Kp->pk); free(Kp);
}

void ora_keys_secret(const ora_keys *Kp, i64 *s) { memcpy(s, Kp->s, Kp->P->n * sizeof(i64)); }

static const ora_swk *find_swk(const ora_keys *Kp, u32 g) {
    for (int w = 0; w < Kp->nswk; w++) if (Kp->swk[w].g == g) return &Kp->swk[w];
    return NULL;
}

int ora_circuit_galois(const ora_params *P, u32 Nr, int what, u32 *out);

/* ORA_OK when the keys hold every rotation key that the circuits `what` (the
 * bits of ora_circuit_galois) need on N values; the circuits assume them */
static int need_keys(const ora_keys *Kp, u32 N, int what) {
    u32 g[256];
    int c = ora_circuit_galois(Kp->P, N, what, g);
    for (int i = 0; i < c; i++)
        if (!find_swk(Kp, g[i])) return ORA_E_INVALID;
    return ORA_OK;
}

/* ---------------- encryption / decryption ---------------- */
ora_ct *ora_encrypt(const ora_keys *Kp, const double *z, u32 count, int level, const u8 seed[32], int *status) {
    const ora_params *P = Kp->P;
    u64 n = P->n;
    if (level < 0 || level > Kp->lmax) { if (status) *status = ORA_E_DEPTH; return NULL; }
    i64 *m = (i64 *)malloc(n * sizeof(i64));
    int st = ora_encode(P, z, count, P->scale[level], m);
    if (st != ORA_OK) { free(m); if (status) *status = st; return NULL; }
    i64 *u = (i64 *)malloc(n * sizeof(i64)), *e0 = (i64 *)malloc(n * sizeof(i64)), *e1 = (i64 *)malloc(n * sizeof(i64));
    { stream_t s; stream_init(&s, seed, PUR_ENC_U, 0); for (u64 i = 0; i < n; i++) u[i] = samp_ternary(&s); }
    { stream_t s; stream_init(&s, seed, PUR_ENC_E0, 0); for (u64 i = 0; i < n; i++) e0[i] = samp_cbd21(&s); }
    { stream_t s; stream_init(&s, seed, PUR_ENC_E1, 0); for (u64 i = 0; i < n; i++) e1[i] = samp_cbd21(&s); }
    ora_ct *c = ct_new(P, level);
    #pragma omp parallel for schedule(dynamic)
    for (int t = 0; t <= level; t++) {
        u64 q = P->mod[t];
        u64 *ul = (u64 *)malloc(n * 8);
        for (u64 i = 0; i < n; i++) ul[i] = red_i64(u[i], q);
        u64 *c0 = LIMB(ct_poly(c, 0), t, n), *c1 = LIMB(ct_poly(c, 1), t, n);
        ring_mul_limb(ul, LIMB(Kp->pk, t, n), c0, P, t);
        ring_mul_limb(ul, LIMB(Kp->pk, Kp->lmax + 1 + t, n), c1, P, t);
        for (u64 i = 0; i < n; i++) {
            c0[i] = addm(c0[i], addm(red_i64(e0[i], q), red_i64(m[i], q), q), q);
            c1[i] = addm(c1[i], red_i64(e1[i], q), q);
        }
        free(ul);
    }
    free(m); free(u); free(e0); free(e1);
    if (status) *status = ORA_OK;
    return c;
}

/* message = c0 + c1*s taken mod q_0 and centred (valid while |m| < q_0/2) */
void ora_decrypt_coeffs(const ora_keys *Kp, const ora_ct *c, i64 *m) {
    const ora_params *P = Kp->P;
    u64 n = P->n, q = P->mod[0];
    u64 *sl = (u64 *)malloc(n * 8), *x = (u64 *)malloc(n * 8);
    for (u64 i = 0; i < n; i++) sl[i] = red_i64(Kp->s[i], q);
    ring_mul_limb(LIMB(ct_poly(c, 1), 0, n), sl, x, P, 0);
    for (u64 i = 0; i < n; i++) {
        u64 v = addm(x[i], LIMB(ct_poly(c, 0), 0, n)[i], q);
        m[i] = v > q / 2 ? -(i64)(q - v) : (i64)v;
    }
    free(sl); free(x);
}

void ora_decrypt(const ora_keys *Kp, const ora_ct *c, double *z, u32 count) {
    i64 *m = (i64 *)malloc(Kp->P->n * sizeof(i64));
    ora_decrypt_coeffs(Kp, c, m);
    ora_decode(Kp->P, m, Kp->P->scale[c->level], count, z);
    free(m);
}

/* ------------------------------------------------------------------ */
/* base conversion, key switching, rescale                             */
/* ------------------------------------------------------------------ */
/* Fast base conversion of one coefficient vector set x (residues mod src[0..ns))
 * to modulus t:  sum_i [x_i * (S/s_i)^{-1}]_{s_i} * (S/s_i mod t)  mod t. */
static void bconv(const u64 *const *x, const u64 *src, int ns, u64 t, u64 *out, u64 n) {
    u64 hinv[ORA_MAXMOD], hmod[ORA_MAXMOD];
    for (int i = 0; i < ns; i++) {
        u64 si = src[i], a = 1 % si, b = 1 % t;
        for (int k = 0; k < ns; k++) if (k != i) { a = mulm(a, src[k] % si, si); b = mulm(b, src[k] % t, t); }
        hinv[i] = invm(a, si); hmod[i] = b;
    }
    for (u64 c = 0; c < n; c++) {
        u64 acc = 0;
        for (int i = 0; i < ns; i++) acc = addm(acc, mulm(mulm(x[i][c], hinv[i], src[i]) % t, hmod[i], t), t);
        out[c] = acc;
    }
}

/* ModDown's base conversion from P = p_0 ... p_{K-1} to t with the overflow
 * removed.  With y_i = [x_i (P/p_i)^{-1}]_{p_i}, the sum S = sum_i y_i (P/p_i)
 * equals (X mod P) + u P for the integer u = floor(sum_i y_i / p_i) in
 * [0, K): the fast conversion's excess.  Uncorrected, u has mean about
 * (K - 1)/2 in every coefficient of both key-switch outputs; the c1 part's
 * bias, times the secret, puts a systematic error of about
 * (K/2) |s(zeta_0)| (2n/pi) / D into slot 0 (the slot whose root lies
 * closest to 1) after every key switch.  u is computed as the floor of the
 * IEEE double sum of y_i * (1/p_i), i = 0 .. K-1 in order, no fused
 * operations (the result can differ from the exact floor only when
 * X mod P lies within about K^2 2^-52 P of a multiple of P), and u P is
 * subtracted: the conversion then returns X mod P itself. */
static void bconv_exact(const u64 *const *x, const u64 *src, int ns, u64 t, u64 *out, u64 n) {
    u64 hinv[ORA_MAXMOD], hmod[ORA_MAXMOD], pmod = 1 % t;
    double rinv[ORA_MAXMOD];
    for (int i = 0; i < ns; i++) {
        u64 si = src[i], a = 1 % si, b = 1 % t;
        for (int k = 0; k < ns; k++) if (k != i) { a = mulm(a, src[k] % si, si); b = mulm(b, src[k] % t, t); }
        hinv[i] = invm(a, si); hmod[i] = b;
        rinv[i] = 1.0 / (double)si;
        pmod = mulm(pmod, si % t, t);
    }
    for (u64 c = 0; c < n; c++) {
        u64 acc = 0;
        double v = 0.0;
        for (int i = 0; i < ns; i++) {
            const u64 y = mulm(x[i][c], hinv[i], src[i]);
            const double f = (double)y * rinv[i];
            v = v + f;
            acc = addm(acc, mulm(y % t, hmod[i], t), t);
        }
        const u64 u = (u64)floor(v);
        out[c] = subm(acc, mulm(u % t, pmod, t), t);
    }
}

/* pin helper: x given as ns limbs of n residues */
void ora_bconv(const u64 *x, const u64 *src, int ns, u64 t, u64 n, u64 *out) {
    const u64 *ptr[ORA_MAXMOD];
    for (int i = 0; i < ns; i++) ptr[i] = x + (size_t)i * n;
    bconv(ptr, src, ns, t, out, n);
}

/* key switch of d (coefficient domain, limbs 0..level) with key w -> (kb, ka), coefficient domain */
/* ModDown rounds: floor((X + (P - 1)/2) / P) = round(X / P), the base
 * conversion's overflow removed (bconv_exact).  This adds (P - 1)/2 to every
 * coefficient of x (coefficient domain), given on q_0..q_level then
 * p_0..p_{K-1}; P is odd, so (P - 1)/2 mod m = (P mod m - 1) / 2 mod m. */
static void add_half_P(const ora_params *P, u64 *x, int level) {
    const u64 n = P->n;
    const int K = P->K;
    for (int i = 0; i <= level + K; i++) {
        const u64 m = i <= level ? P->mod[i] : P->mod[P->nq + (i - level - 1)];
        u64 pm = 1 % m;
        for (int k = 0; k < K; k++) pm = mulm(pm, P->mod[P->nq + k] % m, m);
        const u64 h = mulm(subm(pm, 1 % m, m), invm(2 % m, m), m);
        u64 *xl = LIMB(x, i, n);
        for (u64 c = 0; c < n; c++) xl[c] = addm(xl[c], h, m);
    }
}

static void keyswitch(const ora_keys *Kp, const ora_swk *w, const u64 *d, int level, u64 *kb, u64 *ka) {
    const ora_params *P = Kp->P;
    u64 n = P->n; int lmax = Kp->lmax, K = P->K;
    int E = level + 1 + K, Ek = lmax + 1 + K;
    int beta = (level + 1 + P->alpha - 1) / P->alpha;
    u64 *accb = (u64 *)calloc((size_t)E * n, 8), *acca = (u64 *)calloc((size_t)E * n, 8);
    #pragma omp parallel for schedule(dynamic)
    for (int li = 0; li < E; li++) {
        int mt = li <= level ? li : P->nq + (li - level - 1);
        u64 q = P->mod[mt];
        int kl = key_limb(P, lmax, mt);
        u64 *y = (u64 *)malloc(n * 8);
        for (int j = 0; j < beta; j++) {
            int lo = j * P->alpha, hi = (j + 1) * P->alpha - 1;
            if (hi > level) hi = level;
            if (mt >= lo && mt <= hi) memcpy(y, LIMB(d, mt, n), n * 8);
            else {
                const u64 *ptr[ORA_MAXMOD]; u64 src[ORA_MAXMOD];
                for (int i = lo; i <= hi; i++) { ptr[i - lo] = LIMB(d, i, n); src[i - lo] = P->mod[i]; }
                bconv(ptr, src, hi - lo + 1, q, y, n);
            }
            ntt_fwd(y, n, q, P->psi[mt]);
            const u64 *eb = LIMB(w->d, ((size_t)j * 2 + 0) * Ek + kl, n);
            const u64 *ea = LIMB(w->d, ((size_t)j * 2 + 1) * Ek + kl, n);
            u64 *ob = LIMB(accb, li, n), *oa = LIMB(acca, li, n);
            for (u64 i = 0; i < n; i++) {
                ob[i] = addm(ob[i], mulm(y[i], eb[i], q), q);
                oa[i] = addm(oa[i], mulm(y[i], ea[i], q), q);
            }
        }
        ntt_inv(LIMB(accb, li, n), n, q, P->psi[mt]);
        ntt_inv(LIMB(acca, li, n), n, q, P->psi[mt]);
        free(y);
    }
    /* ModDown: (x_Q - [X mod P]_{q_i}) * P^{-1} mod q_i, X mod P from the exact conversion */
    u64 psrc[ORA_MAXMOD];
    for (int k = 0; k < K; k++) psrc[k] = P->mod[P->nq + k];
    for (int pol = 0; pol < 2; pol++) {
        u64 *acc = pol == 0 ? accb : acca, *out = pol == 0 ? kb : ka;
        add_half_P(P, acc, level);
        const u64 *ptr[ORA_MAXMOD];
        for (int k = 0; k < K; k++) ptr[k] = LIMB(acc, level + 1 + k, n);
        #pragma omp parallel for schedule(dynamic)
        for (int i = 0; i <= level; i++) {
            u64 q = P->mod[i], pinv = 1 % q;
            for (int k = 0; k < K; k++) pinv = mulm(pinv, psrc[k] % q, q);
            pinv = invm(pinv, q);
            u64 *conv = (u64 *)malloc(n * 8);
            bconv_exact(ptr, psrc, K, q, conv, n);
            for (u64 c = 0; c < n; c++) LIMB(out, i, n)[c] = mulm(subm(LIMB(acc, i, n)[c], conv[c], q), pinv, q);
            free(conv);
        }
    }
    free(accb); free(acca);
}

/* pin helper: ModDown of one polynomial given on (q_0..q_level, p_0..p_{K-1}) */
void ora_moddown(const ora_params *P, int level, const u64 *x_in, u64 *out) {
    u64 n = P->n; int K = P->K;
    u64 *x = (u64 *)malloc((size_t)(level + 1 + K) * n * 8);
    memcpy(x, x_in, (size_t)(level + 1 + K) * n * 8);
    add_half_P(P, x, level);
    u64 psrc[ORA_MAXMOD]; const u64 *ptr[ORA_MAXMOD];
    for (int k = 0; k < K; k++) { psrc[k] = P->mod[P->nq + k]; ptr[k] = LIMB(x, level + 1 + k, n); }
    for (int i = 0; i <= level; i++) {
        u64 q = P->mod[i], pinv = 1 % q;
        for (int k = 0; k < K; k++) pinv = mulm(pinv, psrc[k] % q, q);
        pinv = invm(pinv, q);
        u64 *conv = (u64 *)malloc(n * 8);
        bconv_exact(ptr, psrc, K, q, conv, n);
        for (u64 c = 0; c < n; c++) LIMB(out, i, n)[c] = mulm(subm(LIMB(x, i, n)[c], conv[c], q), pinv, q);
        free(conv);
    }
    free(x);
}

/* rounding rescale of one polynomial (limbs 0..level) -> limbs 0..level-1:
 * floor((X + (q_l - 1)/2) / q_l), i.e. (X - v) / q_l with v the residue of X
 * mod q_l taken in (-q_l/2, q_l/2).  A floor would leave every coefficient
 * about 1/2 low, and such a constant coefficient bias b shows in slot k as
 * 2b / (1 - zeta_k), largest in slot 0. */
static void rescale_poly(const ora_params *P, const u64 *x, int level, u64 *out) {
    u64 n = P->n, ql = P->mod[level];
    const u64 *xl = LIMB(x, level, n);
    #pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < level; i++) {
        u64 q = P->mod[i], inv = invm(ql % q, q), qlq = ql % q;
        for (u64 c = 0; c < n; c++) {
            u64 v = xl[c] % q;
            if (xl[c] > ql / 2) v = subm(v, qlq, q);   /* the residue minus q_l */
            LIMB(out, i, n)[c] = mulm(subm(LIMB(x, i, n)[c], v, q), inv, q);
        }
    }
}
void ora_rescale_poly(const ora_params *P, const u64 *x, int level, u64 *out) { rescale_poly(P, x, level, out); }

/* ------------------------------------------------------------------ */
/* homomorphic operations                                              */
/* ------------------------------------------------------------------ */
ora_ct *ora_rescale(const ora_ct *a) {
    ora_ct *c = ct_new(a->P, a->level - 1);
    for (int p = 0; p < 2; p++) rescale_poly(a->P, ct_poly(a, p), a->level, ct_poly(c, p));
    return c;
}

ora_ct *ora_drop(const ora_ct *a, int level) {
    ora_ct *c = ct_new(a->P, level);
    u64 n = a->P->n;
    for (int p = 0; p < 2; p++) memcpy(ct_poly(c, p), ct_poly(a, p), (size_t)(level + 1) * n * 8);
    return c;
}

ora_ct *ora_add(const ora_ct *a, const ora_ct *b) {
    if (a->level != b->level) return NULL;
    ora_ct *c = ct_new(a->P, a->level);
    u64 n = a->P->n;
    for (int p = 0; p < 2; p++)
        for (int t = 0; t <= a->level; t++) {
            u64 q = a->P->mod[t];
            for (u64 i = 0; i < n; i++)
                LIMB(ct_poly(c, p), t, n)[i] = addm(LIMB(ct_poly(a, p), t, n)[i], LIMB(ct_poly(b, p), t, n)[i], q);
        }
    return c;
}

ora_ct *ora_sub(const ora_ct *a, const ora_ct *b) {
    if (a->level != b->level) return NULL;
    ora_ct *c = ct_new(a->P, a->level);
    u64 n = a->P->n;
    for (int p = 0; p < 2; p++)
        for (int t = 0; t <= a->level; t++) {
            u64 q = a->P->mod[t];
            for (u64 i = 0; i < n; i++)
                LIMB(ct_poly(c, p), t, n)[i] = subm(LIMB(ct_poly(a, p), t, n)[i], LIMB(ct_poly(b, p), t, n)[i], q);
        }
    return c;
}

/* add the constant c (every slot): round(c * D_l) on the constant coefficient of c0 */
ora_ct *ora_add_const(const ora_ct *a, double cst) {
    ora_ct *c = ct_copy(a);
    i64 K = llround(cst * a->P->scale[a->level]);
    u64 n = a->P->n;
    for (int t = 0; t <= a->level; t++) {
        u64 q = a->P->mod[t];
        LIMB(ct_poly(c, 0), t, n)[0] = addm(LIMB(ct_poly(c, 0), t, n)[0], red_i64(K, q), q);
    }
    return c;
}

/* multiply by the signed integer K, no rescale */
static ora_ct *mul_int(const ora_ct *a, i64 K) {
    ora_ct *c = ct_copy(a);
    u64 n = a->P->n;
    for (int p = 0; p < 2; p++)
        for (int t = 0; t <= a->level; t++) {
            u64 q = a->P->mod[t], k = red_i64(K, q);
            u64 *x = LIMB(ct_poly(c, p), t, n);
            for (u64 i = 0; i < n; i++) x[i] = mulm(x[i], k, q);
        }
    return c;
}

/* c * x brought to level `target` < level(x): drop to target+1 limbs, multiply by
 * round(c * D_target * q_{target+1} / D_level(x)), rescale by q_{target+1}. */
ora_ct *ora_cmul_to(const ora_ct *a, double cst, int target, int *status) {
    const ora_params *P = a->P;
    if (target < 0 || target >= a->level) { if (status) *status = ORA_E_DEPTH; return NULL; }
    double v = ((cst * P->scale[target]) * (double)P->mod[target + 1]) / P->scale[a->level];
    i64 K = llround(v);
    ora_ct *d = ora_drop(a, target + 1);
    ora_ct *m = mul_int(d, K);
    ora_ct *r = ora_rescale(m);
    ora_ct_free(d); ora_ct_free(m);
    if (status) *status = ORA_OK;
    return r;
}

/* slot-wise product with a plaintext holding z on slots [0,count) at scale D_l, then rescale */
ora_ct *ora_mul_plain(const ora_ct *a, const double *z, u32 count, int *status) {
    const ora_params *P = a->P;
    u64 n = P->n;
    if (a->level < 1) { if (status) *status = ORA_E_DEPTH; return NULL; }
    i64 *m = (i64 *)malloc(n * sizeof(i64));
    int st = ora_encode(P, z, count, P->scale[a->level], m);
    if (st != ORA_OK) { free(m); if (status) *status = st; return NULL; }
    ora_ct *c = ct_new(P, a->level);
    #pragma omp parallel for schedule(dynamic)
    for (int t = 0; t <= a->level; t++) {
        u64 q = P->mod[t];
        u64 *ml = (u64 *)malloc(n * 8);
        for (u64 i = 0; i < n; i++) ml[i] = red_i64(m[i], q);
        for (int p = 0; p < 2; p++) ring_mul_limb(LIMB(ct_poly(a, p), t, n), ml, LIMB(ct_poly(c, p), t, n), P, t);
        free(ml);
    }
    free(m);
    ora_ct *r = ora_rescale(c);
    ora_ct_free(c);
    if (status) *status = ORA_OK;
    return r;
}

/* add a plaintext holding z on slots [0,count) at the ciphertext's scale */
ora_ct *ora_add_plain(const ora_ct *a, const double *z, u32 count, int *status) {
    const ora_params *P = a->P;
    u64 n = P->n;
    i64 *m = (i64 *)malloc(n * sizeof(i64));
    int st = ora_encode(P, z, count, P->scale[a->level], m);
    if (st != ORA_OK) { free(m); if (status) *status = st; return NULL; }
    ora_ct *c = ct_copy(a);
    for (int t = 0; t <= a->level; t++) {
        u64 q = P->mod[t];
        u64 *x = LIMB(ct_poly(c, 0), t, n);
        for (u64 i = 0; i < n; i++) x[i] = addm(x[i], red_i64(m[i], q), q);
    }
    free(m);
    if (status) *status = ORA_OK;
    return c;
}

/* ct * ct: tensor, relinearise with the s^2 key, rescale */
ora_ct *ora_mul(const ora_keys *Kp, const ora_ct *a, const ora_ct *b, int *status) {
    const ora_params *P = a->P;
    u64 n = P->n; int l = a->level;
    if (b->level != l || l < 1 || l > Kp->lmax) { if (status) *status = ORA_E_DEPTH; return NULL; }
    u64 *d0 = (u64 *)malloc((size_t)(l + 1) * n * 8), *d1 = (u64 *)malloc((size_t)(l + 1) * n * 8),
        *d2 = (u64 *)malloc((size_t)(l + 1) * n * 8);
    #pragma omp parallel for schedule(dynamic)
    for (int t = 0; t <= l; t++) {
        u64 q = P->mod[t];
        u64 *A0 = (u64 *)malloc(n * 8), *A1 = (u64 *)malloc(n * 8), *B0 = (u64 *)malloc(n * 8), *B1 = (u64 *)malloc(n * 8);
        memcpy(A0, LIMB(ct_poly(a, 0), t, n), n * 8); memcpy(A1, LIMB(ct_poly(a, 1), t, n), n * 8);
        memcpy(B0, LIMB(ct_poly(b, 0), t, n), n * 8); memcpy(B1, LIMB(ct_poly(b, 1), t, n), n * 8);
        ntt_fwd(A0, n, q, P->psi[t]); ntt_fwd(A1, n, q, P->psi[t]);
        ntt_fwd(B0, n, q, P->psi[t]); ntt_fwd(B1, n, q, P->psi[t]);
        u64 *x0 = LIMB(d0, t, n), *x1 = LIMB(d1, t, n), *x2 = LIMB(d2, t, n);
        for (u64 i = 0; i < n; i++) {
            x0[i] = mulm(A0[i], B0[i], q);
            x1[i] = addm(mulm(A0[i], B1[i], q), mulm(A1[i], B0[i], q), q);
            x2[i] = mulm(A1[i], B1[i], q);
        }
        ntt_inv(x0, n, q, P->psi[t]); ntt_inv(x1, n, q, P->psi[t]); ntt_inv(x2, n, q, P->psi[t]);
        free(A0); free(A1); free(B0); free(B1);
    }
    u64 *kb = (u64 *)malloc((size_t)(l + 1) * n * 8), *ka = (u64 *)malloc((size_t)(l + 1) * n * 8);
    keyswitch(Kp, find_swk(Kp, 0), d2, l, kb, ka);
    ora_ct *c = ct_new(P, l);
    for (int t = 0; t <= l; t++) {
        u64 q = P->mod[t];
        for (u64 i = 0; i < n; i++) {
            LIMB(ct_poly(c, 0), t, n)[i] = addm(LIMB(d0, t, n)[i], LIMB(kb, t, n)[i], q);
            LIMB(ct_poly(c, 1), t, n)[i] = addm(LIMB(d1, t, n)[i], LIMB(ka, t, n)[i], q);
        }
    }
    free(d0); free(d1); free(d2); free(kb); free(ka);
    ora_ct *r = ora_rescale(c);
    ora_ct_free(c);
    if (status) *status = ORA_OK;
    return r;
}

/* left rotation of the slot vector by k (new[j] = old[j+k]), Galois element 5^k mod 2n */
static u32 gal_left(const ora_params *P, u64 k) { return (u32)powm(5, k % (P->n / 2), 2 * P->n); }

ora_ct *ora_apply_galois(const ora_keys *Kp, const ora_ct *a, u32 g, int *status) {
    const ora_params *P = a->P;
    u64 n = P->n; int l = a->level;
    const ora_swk *w = find_swk(Kp, g);
    if (!w || l > Kp->lmax) { if (status) *status = ORA_E_INVALID; return NULL; }
    u64 *c0 = (u64 *)malloc((size_t)(l + 1) * n * 8), *c1 = (u64 *)malloc((size_t)(l + 1) * n * 8);
    for (int t = 0; t <= l; t++) {
        automorph_limb(LIMB(ct_poly(a, 0), t, n), LIMB(c0, t, n), n, P->mod[t], g);
        automorph_limb(LIMB(ct_poly(a, 1), t, n), LIMB(c1, t, n), n, P->mod[t], g);
    }
    u64 *kb = (u64 *)malloc((size_t)(l + 1) * n * 8), *ka = (u64 *)malloc((size_t)(l + 1) * n * 8);
    keyswitch(Kp, w, c1, l, kb, ka);
    ora_ct *c = ct_new(P, l);
    for (int t = 0; t <= l; t++) {
        u64 q = P->mod[t];
        for (u64 i = 0; i < n; i++) {
            LIMB(ct_poly(c, 0), t, n)[i] = addm(LIMB(c0, t, n)[i], LIMB(kb, t, n)[i], q);
            LIMB(ct_poly(c, 1), t, n)[i] = LIMB(ka, t, n)[i];
        }
    }
    free(c0); free(c1); free(kb); free(ka);
    if (status) *status = ORA_OK;
    return c;
}

ora_ct *ora_rotate(const ora_keys *Kp, const ora_ct *a, i64 k, int *status) {
    i64 h = (i64)(Kp->P->n / 2);
    i64 kk = ((k % h) + h) % h;
    if (kk == 0) { if (status) *status = ORA_OK; return ct_copy(a); }
    return ora_apply_galois(Kp, a, gal_left(Kp->P, (u64)kk), status);
}

/* ------------------------------------------------------------------ */
/* matrix operations (section 2.3, Algorithms TransR/TransC, App. A)   */
/* An N x N matrix occupies slots [0, N^2) row by row.                 */
/* ------------------------------------------------------------------ */
static void replace(ora_ct **x, ora_ct *y) { ora_ct_free(*x); *x = y; }

static int ilog2(u32 N) { int r = 0; while ((1u << r) < N) r++; return r; }

/* X + (X rotated left by k), or right by k when k < 0 */
static ora_ct *add_rot(const ora_keys *Kp, const ora_ct *X, i64 k, int *st) {
    ora_ct *r = ora_rotate(Kp, X, k, st);
    if (!r) return NULL;
    ora_ct *s = ora_add(X, r);
    ora_ct_free(r);
    return s;
}

/* mask keeping row `row` (slots [row*N, row*N+N)) */
static ora_ct *mask_row(const ora_ct *X, u32 N, u32 row, int *st) {
    double *z = (double *)calloc((size_t)N * N, sizeof(double));
    for (u32 j = 0; j < N; j++) z[row * N + j] = 1.0;
    ora_ct *r = ora_mul_plain(X, z, N * N, st);
    free(z);
    return r;
}
/* mask keeping column `col` (slots i*N+col) */
static ora_ct *mask_col(const ora_ct *X, u32 N, u32 col, int *st) {
    double *z = (double *)calloc((size_t)N * N, sizeof(double));
    for (u32 i = 0; i < N; i++) z[i * N + col] = 1.0;
    ora_ct *r = ora_mul_plain(X, z, N * N, st);
    free(z);
    return r;
}

/* TransR: row vector -> column vector; right rotations by N(N-1)/2^i, then MaskC(.,0) */
ora_ct *ora_trans_r(const ora_keys *Kp, const ora_ct *V, u32 N, int *st) {
    ora_ct *X = ct_copy(V);
    for (int i = 1; i <= ilog2(N); i++) replace(&X, add_rot(Kp, X, -(i64)((u64)N * (N - 1) >> i), st));
    replace(&X, mask_col(X, N, 0, st));
    return X;
}
/* TransC: column vector -> row vector; left rotations by N(N-1)/2^i, then MaskR(.,0) */
ora_ct *ora_trans_c(const ora_keys *Kp, const ora_ct *V, u32 N, int *st) {
    ora_ct *X = ct_copy(V);
    for (int i = 1; i <= ilog2(N); i++) replace(&X, add_rot(Kp, X, (i64)((u64)N * (N - 1) >> i), st));
    replace(&X, mask_row(X, N, 0, st));
    return X;
}
/* SumR: rows summed into row 0; left rotations by N*2^i, then MaskR(.,0) */
ora_ct *ora_sum_r(const ora_keys *Kp, const ora_ct *V, u32 N, int *st) {
    ora_ct *X = ct_copy(V);
    for (int i = 0; i < ilog2(N); i++) replace(&X, add_rot(Kp, X, (i64)N << i, st));
    replace(&X, mask_row(X, N, 0, st));
    return X;
}
/* SumC: columns summed into column 0; left rotations by 2^i, then MaskC(.,0) */
ora_ct *ora_sum_c(const ora_keys *Kp, const ora_ct *V, u32 N, int *st) {
    ora_ct *X = ct_copy(V);
    for (int i = 0; i < ilog2(N); i++) replace(&X, add_rot(Kp, X, (i64)1 << i, st));
    replace(&X, mask_col(X, N, 0, st));
    return X;
}
/* ReplR: row 0 copied to every row; right rotations by N*2^i */
ora_ct *ora_repl_r(const ora_keys *Kp, const ora_ct *V, u32 N, int *st) {
    ora_ct *X = ct_copy(V);
    for (int i = 0; i < ilog2(N); i++) replace(&X, add_rot(Kp, X, -((i64)N << i), st));
    return X;
}
/* ReplC: column 0 copied to every column; right rotations by 2^i */
ora_ct *ora_repl_c(const ora_keys *Kp, const ora_ct *V, u32 N, int *st) {
    ora_ct *X = ct_copy(V);
    for (int i = 0; i < ilog2(N); i++) replace(&X, add_rot(Kp, X, -((i64)1 << i), st));
    return X;
}

/* ------------------------------------------------------------------ */
/* comparison: composite of the odd degree-7 polynomials f and g       */
/* (section 2.2):  Cmp(x, y) = (f^{d_f}(g^{d_g}(x - y)) + 1) / 2        */
/* ------------------------------------------------------------------ */
static const double F_COEF[4] = {35.0 / 16, -35.0 / 16, 21.0 / 16, -5.0 / 16};
static const double G_COEF[4] = {4589.0 / 1024, -16577.0 / 1024, 25614.0 / 1024, -12860.0 / 1024};
/* The minimax composite (section 2.2 names composite minimax approximations
 * of the sign function as the alternative to f and g): stage 0 is the odd
 * degree-7 polynomial closest to 1 in the maximum norm on [2^-8.5, 1], stage
 * s the one closest to 1 on the interval stage s-1 maps that onto.  Each
 * equioscillates on its interval at 5 points; the errors are 0.968, 0.827,
 * 0.362, 9.8e-3 and 5.1e-9.  Coefficients of x, x^3, x^5, x^7. */
#define MM_STAGES 5
static const double MM_COEF[MM_STAGES][4] = {
    {11.626630381861787, -68.36534054680979, 126.44790262989271, -69.67707957286088},
    {5.38484717173034, -7.907363201737443, 3.7393070660732937, -0.5295271268765817},
    {3.8547436306459173, -5.358791130620638, 2.7473565274453287, -0.4363096838044091},
    {2.363269725894833, -2.5537068630909263, 1.5095093062451124, -0.32798232661912397},
    {2.1876161909909757, -2.187742945230383, 1.3126373118789916, -0.3125105627390891},
};

/* a1 x + a3 x^3 + a5 x^5 + a7 x^7 (a7 != 0) at depth 3 with four products:
 *   y = x*x, t = (a7 x)*y = a7 x^3, y2 = y*y, h = y2*(t + a5 x) = a7 x^7 + a5 x^5,
 *   p = h + (a3/a7) t + a1 x, the last two terms brought to level l-3 by cmul_to
 * (a3 x^3 comes from t by a constant product instead of a fifth ciphertext
 * product). */
ora_ct *ora_poly7(const ora_keys *Kp, const ora_ct *x, const double a[4], int *st) {
    int l = x->level;
    if (l < 3) { *st = ORA_E_DEPTH; return NULL; }
    if (a[3] == 0.0) { *st = ORA_E_INVALID; return NULL; }
    ora_ct *y = ora_mul(Kp, x, x, st);
    ora_ct *u7 = ora_cmul_to(x, a[3], l - 1, st);
    ora_ct *t = ora_mul(Kp, u7, y, st);
    ora_ct *y2 = ora_mul(Kp, y, y, st);
    ora_ct *u5 = ora_cmul_to(x, a[2], l - 2, st);
    ora_ct *w = ora_add(t, u5);
    ora_ct *h = ora_mul(Kp, y2, w, st);
    ora_ct *v3 = ora_cmul_to(t, a[1] / a[3], l - 3, st);
    ora_ct *v1 = ora_cmul_to(x, a[0], l - 3, st);
    ora_ct *s1 = ora_add(h, v3);
    ora_ct *p = ora_add(s1, v1);
    ora_ct_free(y); ora_ct_free(u7); ora_ct_free(t); ora_ct_free(y2); ora_ct_free(u5); ora_ct_free(w);
    ora_ct_free(h); ora_ct_free(v3); ora_ct_free(v1); ora_ct_free(s1);
    return p;
}

/* ------------------------------------------------------------------ */
/* Chebyshev comparator (section 2.2): Eq. (1) as a function of         */
/* d = x - y, interpolated on [-1, 1] at the 2M = 2^(D-1) Chebyshev      */
/* nodes (degree 2M - 1), evaluated with the Paterson-Stockmeyer         */
/* algorithm in the Chebyshev basis in D levels.                          */
/* ------------------------------------------------------------------ */
/* Interpolation coefficients: c_k = (2/2M) sum_j f(x_j) T_k(x_j) over the
 * nodes x_j = cos(pi (j + 1/2) / 2M), halved for k = 0.  f is 1 on the M
 * positive nodes and 0 on the others, so the sum is a geometric cosine sum:
 * c_0 = 1/2, c_k = 0 for even k > 0, and for odd k
 *   c_k = (-1)^((k-1)/2) / (2M sin(pi k / 4M)).
 * Evaluated in binary128 and rounded once to double. */
void ora_cheb_step_coeffs(int D, double *c) {
    const long M = 1L << (D - 2);
    c[0] = 0.5;
    for (long k = 1; k < 2 * M; k++) {
        if ((k & 1) == 0) { c[k] = 0.0; continue; }
        __float128 den = (__float128)(2 * M) * sinq(M_PIq * (__float128)k / (__float128)(4 * M));
        __float128 v = (((k - 1) / 2) & 1 ? -1.0Q : 1.0Q) / den;
        c[k] = (double)v;
    }
}

/* x brought down to `level` (a copy when it is already there) */
static ora_ct *align_to(const ora_ct *x, int level, int *st) {
    return x->level == level ? ct_copy(x) : ora_cmul_to(x, 1.0, level, st);
}

/* 2 a b - s (s = NULL: the constant 1), a and b first brought to one level */
static ora_ct *cheb_step(const ora_keys *Kp, const ora_ct *a, const ora_ct *b, const ora_ct *s, int *st) {
    int lv = a->level < b->level ? a->level : b->level;
    ora_ct *A = align_to(a, lv, st), *B = align_to(b, lv, st);
    ora_ct *pr = ora_mul(Kp, A, B, st);
    ora_ct *p2 = mul_int(pr, 2);
    ora_ct *out;
    if (s) {
        ora_ct *S = align_to(s, p2->level, st);
        out = ora_sub(p2, S);
        ora_ct_free(S);
    } else {
        out = ora_add_const(p2, -1.0);
    }
    ora_ct_free(A); ora_ct_free(B); ora_ct_free(pr); ora_ct_free(p2);
    return out;
}

typedef struct {
    const ora_keys *Kp;
    int k;           /* baby steps T_1 .. T_{k-1}, all at level lb */
    int lb;
    ora_ct **Tb;     /* [k] baby steps brought to level lb (index 0 unused) */
    ora_ct **G;      /* giant steps G_r = T_{k 2^r} */
} cheb_ctx;

/* sum_{i<n} c_i T_i for n = k 2^r.  r = 0: a linear combination of the baby
 * steps, sum_i round(c_i D_{lb-1} q_lb / D_lb) T_i over T_1 and every i with
 * c_i != 0, one rescale, then + c_0.  r > 0: with K = k 2^(r-1), the
 * division p = q T_K + s of the Chebyshev identity
 * T_{K+j} = 2 T_j T_K - T_{K-j}:
 *   q_0 = c_K, q_j = 2 c_{K+j};  s_0 = c_0, s_i = c_i - c_{2K-i}  (0 < i, j < K),
 * then p = q(x) * G_{r-1} + s(x), each factor brought to the other's level. */
static ora_ct *cheb_rec(const cheb_ctx *X, const double *c, int r, int *st) {
    const ora_params *P = X->Kp->P;
    if (r == 0) {
        const int t = X->lb - 1;
        ora_ct *acc = NULL;
        for (int i = 1; i < X->k; i++) {
            if (i > 1 && c[i] == 0.0) continue;
            i64 K = llround(((c[i] * P->scale[t]) * (double)P->mod[t + 1]) / P->scale[X->lb]);
            ora_ct *term = mul_int(X->Tb[i], K);
            if (acc) { replace(&acc, ora_add(acc, term)); ora_ct_free(term); }
            else acc = term;
        }
        ora_ct *res = ora_rescale(acc);
        ora_ct_free(acc);
        replace(&res, ora_add_const(res, c[0]));
        return res;
    }
    const int K = X->k << (r - 1);
    double *q = (double *)malloc(K * sizeof(double)), *s = (double *)malloc(K * sizeof(double));
    q[0] = c[K];
    s[0] = c[0];
    for (int j = 1; j < K; j++) {
        q[j] = 2.0 * c[K + j];
        s[j] = c[j] - c[2 * K - j];
    }
    ora_ct *Q = cheb_rec(X, q, r - 1, st);
    ora_ct *S = cheb_rec(X, s, r - 1, st);
    ora_ct *Ga = align_to(X->G[r - 1], Q->level, st);
    ora_ct *pr = ora_mul(X->Kp, Q, Ga, st);
    ora_ct *Sa = align_to(S, pr->level, st);
    ora_ct *out = ora_add(pr, Sa);
    ora_ct_free(Q); ora_ct_free(S); ora_ct_free(Ga); ora_ct_free(pr); ora_ct_free(Sa);
    free(q); free(s);
    return out;
}

int ora_cheb_depth(u32 deg1) { int b = ilog2(deg1); return b + 1; }

/* p(x) = sum_{i < deg1} c_i T_i(x) for deg1 = 2^B (B >= 1), by the
 * Paterson-Stockmeyer algorithm in the Chebyshev basis with k = 2^l baby
 * steps, l = ceil(B/2), and m = B - l giant steps:
 *   T_1 = x, T_{2j} = 2 T_j^2 - 1, T_{2j+1} = 2 T_j T_{j+1} - T_1 (j >= 1),
 *   G_0 = T_k, G_r = 2 G_{r-1}^2 - 1,
 * the baby steps brought to one level before the linear combinations.
 * x at level L leaves at level L - B - 1. */
ora_ct *ora_cheb_eval(const ora_keys *Kp, const ora_ct *x, const double *c, u32 deg1, int *st) {
    const int B = ilog2(deg1);
    if (deg1 < 2 || (1u << B) != deg1) { *st = ORA_E_INVALID; return NULL; }
    if (x->level < B + 1) { *st = ORA_E_DEPTH; return NULL; }
    const int l = (B + 1) / 2, m = B - l, k = 1 << l;
    const int top = m > 0 ? k : k - 1; /* T_k is needed only as G_0 */
    ora_ct **T = (ora_ct **)calloc(k + 1, sizeof(ora_ct *));
    T[1] = ct_copy(x);
    for (int j = 2; j <= top; j++)
        T[j] = (j & 1) ? cheb_step(Kp, T[j / 2], T[j / 2 + 1], T[1], st) : cheb_step(Kp, T[j / 2], T[j / 2], NULL, st);
    cheb_ctx X;
    X.Kp = Kp;
    X.k = k;
    X.lb = x->level - l;
    X.Tb = (ora_ct **)calloc(k, sizeof(ora_ct *));
    for (int i = 1; i < k; i++) X.Tb[i] = align_to(T[i], X.lb, st);
    X.G = (ora_ct **)calloc(m > 0 ? m : 1, sizeof(ora_ct *));
    if (m > 0) {
        X.G[0] = ct_copy(T[k]);
        for (int r = 1; r < m; r++) X.G[r] = cheb_step(Kp, X.G[r - 1], X.G[r - 1], NULL, st);
    }
    ora_ct *p = cheb_rec(&X, c, m, st);
    for (int j = 1; j <= top; j++) ora_ct_free(T[j]);
    for (int i = 1; i < k; i++) ora_ct_free(X.Tb[i]);
    for (int r = 0; r < m; r++) ora_ct_free(X.G[r]);
    free(T); free(X.Tb); free(X.G);
    return p;
}

/* ------------------------------------------------------------------ */
/* comparator dispatch                                                  */
/* ------------------------------------------------------------------ */
/* levels the comparator takes: 3 per degree-7 polynomial of the f/g
 * composite, D for the Chebyshev interpolant */
static int cmp_levels(ora_cmp c) { return c.cheb > 0 ? c.cheb : 3 * (c.dg + c.df + c.mm); }

static int cmp_valid(ora_cmp c) {
    if (c.cheb != 0) return c.dg == 0 && c.df == 0 && c.mm == 0 && c.cheb >= 2 && c.cheb <= 16;
    if (c.mm != 0) return c.dg == 0 && c.df == 0 && c.mm >= 1 && c.mm <= MM_STAGES;
    return c.dg >= 0 && c.df >= 0 && c.dg + c.df >= 1;
}

/* a * Cmp on the difference D.  f/g: a * (f^{d_f}(g^{d_g}(D)) + 1) / 2,
 * the factor a/2 folded into the last polynomial and a/2 added as a
 * constant.  Chebyshev: sum_k (a c_k) T_k(D). */
static ora_ct *cmp_sign_scaled(const ora_keys *Kp, const ora_ct *D, ora_cmp cm, double a, int *st) {
    if (!cmp_valid(cm)) { *st = ORA_E_INVALID; return NULL; }
    if (D->level < cmp_levels(cm)) { *st = ORA_E_DEPTH; return NULL; }
    if (cm.cheb > 0) {
        const u32 deg1 = 1u << (cm.cheb - 1);
        double *c = (double *)malloc(deg1 * sizeof(double));
        ora_cheb_step_coeffs(cm.cheb, c);
        for (u32 i = 0; i < deg1; i++) c[i] = c[i] * a;
        ora_ct *r = ora_cheb_eval(Kp, D, c, deg1, st);
        free(c);
        return r;
    }
    ora_ct *X = ct_copy(D);
    int total = cm.mm > 0 ? cm.mm : cm.dg + cm.df;
    for (int r = 0; r < total; r++) {
        const double *c = cm.mm > 0 ? MM_COEF[r] : (r < cm.dg ? G_COEF : F_COEF);
        double cc[4];
        for (int i = 0; i < 4; i++) cc[i] = (r == total - 1) ? c[i] * (a * 0.5) : c[i];
        replace(&X, ora_poly7(Kp, X, cc, st));
    }
    replace(&X, ora_add_const(X, a * 0.5));
    return X;
}

/* A Chebyshev indicator of degree 2^(D-1) - 1 grows like cosh(n y / sqrt(1 - x^2))
 * at x + iy: the imaginary parts its argument inherits (the comparator's
 * slope amplifies the slots' imaginary noise) must be removed first.  x is
 * projected onto its real part as x + conj(x), conj = sigma_{2n-1}, with the
 * factor 1/2 folded into the scaling that precedes it. */
static ora_ct *plus_conj(const ora_keys *Kp, const ora_ct *x, int *st) {
    ora_ct *c = ora_apply_galois(Kp, x, (u32)(2 * x->P->n - 1), st);
    ora_ct *r = ora_add(x, c);
    ora_ct_free(c);
    return r;
}

ora_ct *ora_cmp_sign(const ora_keys *Kp, const ora_ct *D, ora_cmp cm, int *st) {
    return cmp_sign_scaled(Kp, D, cm, 1.0, st);
}

/* ------------------------------------------------------------------ */
/* Rank (Algorithm 3)                                                  */
/* ------------------------------------------------------------------ */
static int check_N(const ora_params *P, u32 N) {
    if (N < 2 || (N & (N - 1)) || (u64)N * N > P->n / 2) return ORA_E_RANGE;
    return ORA_OK;
}

/* levels consumed by rank: MaskC of TransR, the comparator, MaskR of SumR */
int ora_rank_depth(ora_cmp cm) { return 2 + cmp_levels(cm); }

/* Rank of N values that are not a power of two (section 3.1): the vector is
 * padded with zeros to the next power of two Np and the comparison matrix is
 * masked to its N x N block after the comparison, so the padding takes part
 * in no comparison; one more level. */
static u32 pow2_ceil(u32 N) { u32 p = 1; while (p < N) p <<= 1; return p; }

static int check_N_padded(const ora_params *P, u32 N) {
    u32 Np = pow2_ceil(N);
    if (N < 2 || (u64)Np * Np > P->n / 2) return ORA_E_RANGE;
    return ORA_OK;
}

int ora_rank_depth_n(u32 N, ora_cmp cm, int tie) {
    return ora_rank_depth(cm) + (tie ? 2 : 0) + (pow2_ceil(N) != N ? 1 : 0);
}

/* C restricted to its N x N block in the Np x Np layout */
static ora_ct *block_mask(const ora_ct *C, u32 N, u32 Np, int *st) {
    double *z = (double *)calloc((size_t)Np * Np, sizeof(double));
    for (u32 i = 0; i < N; i++)
        for (u32 j = 0; j < N; j++) z[(size_t)i * Np + j] = 1.0;
    ora_ct *r = ora_mul_plain(C, z, Np * Np, st);
    free(z);
    return r;
}

/* a * C with C = Cmp(V_R, V_C) as an N x N matrix (C[i][j] = Cmp(v_j, v_i)) */
static ora_ct *cmp_matrix_scaled(const ora_keys *Kp, const ora_ct *V, u32 N, ora_cmp cm, double a, int *st) {
    ora_ct *VR = ora_repl_r(Kp, V, N, st);
    ora_ct *T = ora_trans_r(Kp, V, N, st);
    ora_ct *VC = ora_repl_c(Kp, T, N, st);
    ora_ct *VRa = ora_cmul_to(VR, 1.0, VC->level, st);
    ora_ct *D = ora_sub(VRa, VC);
    ora_ct *C = cmp_sign_scaled(Kp, D, cm, a, st);
    ora_ct_free(VR); ora_ct_free(T); ora_ct_free(VC); ora_ct_free(VRa); ora_ct_free(D);
    return C;
}

ora_ct *ora_cmp_matrix(const ora_keys *Kp, const ora_ct *V, u32 N, ora_cmp cm, int *st) {
    return cmp_matrix_scaled(Kp, V, N, cm, 1.0, st);
}

ora_ct *ora_rank(const ora_keys *Kp, const ora_ct *V, u32 N, ora_cmp cm, int *status) {
    int st = check_N_padded(Kp->P, N);
    if (st != ORA_OK) { *status = st; return NULL; }
    if ((st = need_keys(Kp, N, 1)) != ORA_OK) { *status = st; return NULL; }
    if (V->level < ora_rank_depth_n(N, cm, 0)) { *status = ORA_E_DEPTH; return NULL; }
    const u32 Np = pow2_ceil(N);
    ora_ct *C = ora_cmp_matrix(Kp, V, Np, cm, &st);
    if (Np != N) replace(&C, block_mask(C, N, Np, &st));
    ora_ct *S = ora_sum_r(Kp, C, Np, &st);
    double *half = (double *)malloc(N * sizeof(double));
    for (u32 j = 0; j < N; j++) half[j] = 0.5;
    ora_ct *R = ora_add_plain(S, half, N, &st);
    free(half); ora_ct_free(C); ora_ct_free(S);
    *status = st;
    return R;
}

/* Multi-Ciphertext Ranking (section 5, Algorithm Multi-Ciphertext Ranking):
 * v split into L blocks B_1..B_L of b values each (slots [0,b) of separate
 * ciphertexts, one level).  C_{i,j} = Cmp(ReplR(B_i), ReplC(TransR(B_j))) is
 * evaluated for j >= i only; the blocks below the diagonal follow from
 * Equation (3), C_{i,j} = (1 - C_{j,i})^T, taken column-wise:
 *   R_i = TransC(SumC(sum_{j<i} (1 - C_{j,i}))) + SumR(sum_{j>=i} C_{i,j}) + 1/2,
 * where sum_{j<i} (1 - C_{j,i}) is evaluated as (i - 1) - sum_{j<i} C_{j,i}
 * (one constant add).  The SumR term is brought down to the TransC term's
 * level, so every R_i leaves at level(B) - depth. */
int ora_rank_multi_depth(ora_cmp cm) { return 3 + cmp_levels(cm); }

int ora_rank_multi(const ora_keys *Kp, ora_ct *const *Bk, u32 L, u32 b, ora_cmp cm, ora_ct **R) {
    int st = check_N(Kp->P, b);
    if (st != ORA_OK) return st;
    if ((st = need_keys(Kp, b, 4)) != ORA_OK) return st;
    if (L < 1) return ORA_E_INVALID;
    for (u32 i = 0; i < L; i++)
        if (Bk[i]->level != Bk[0]->level) return ORA_E_INVALID;
    if (Bk[0]->level < ora_rank_multi_depth(cm)) return ORA_E_DEPTH;
    ora_ct **VR = (ora_ct **)calloc(L, sizeof(ora_ct *)), **VC = (ora_ct **)calloc(L, sizeof(ora_ct *));
    ora_ct **Cm = (ora_ct **)calloc((size_t)L * L, sizeof(ora_ct *));
    for (u32 i = 0; i < L; i++) {
        VR[i] = ora_repl_r(Kp, Bk[i], b, &st);
        ora_ct *T = ora_trans_r(Kp, Bk[i], b, &st);
        VC[i] = ora_repl_c(Kp, T, b, &st);
        ora_ct_free(T);
    }
    for (u32 i = 0; i < L; i++)
        for (u32 j = i; j < L; j++) {
            ora_ct *VRa = ora_cmul_to(VR[i], 1.0, VC[j]->level, &st);
            ora_ct *D = ora_sub(VRa, VC[j]);
            Cm[i * L + j] = ora_cmp_sign(Kp, D, cm, &st);
            ora_ct_free(VRa); ora_ct_free(D);
        }
    const int lc = Cm[0]->level; /* comparator output level */
    double *half = (double *)malloc(b * sizeof(double));
    for (u32 t = 0; t < b; t++) half[t] = 0.5;
    for (u32 i = 0; i < L; i++) {
        ora_ct *S = ct_copy(Cm[i * L + i]);
        for (u32 j = i + 1; j < L; j++) replace(&S, ora_add(S, Cm[i * L + j]));
        ora_ct *Rr = ora_sum_r(Kp, S, b, &st);
        ora_ct *X = ora_cmul_to(Rr, 1.0, lc - 2, &st);
        if (i > 0) {
            ora_ct *Tc = ct_copy(Cm[0 * L + i]);
            for (u32 j = 1; j < i; j++) replace(&Tc, ora_add(Tc, Cm[j * L + i]));
            ora_ct *nT = mul_int(Tc, -1);
            ora_ct *Y = ora_add_const(nT, (double)i);
            ora_ct *SC = ora_sum_c(Kp, Y, b, &st);
            ora_ct *TC = ora_trans_c(Kp, SC, b, &st);
            replace(&X, ora_add(X, TC));
            ora_ct_free(Tc); ora_ct_free(nT); ora_ct_free(Y); ora_ct_free(SC); ora_ct_free(TC);
        }
        R[i] = ora_add_plain(X, half, b, &st);
        ora_ct_free(S); ora_ct_free(Rr); ora_ct_free(X);
    }
    free(half);
    for (u32 i = 0; i < L; i++) {
        ora_ct_free(VR[i]); ora_ct_free(VC[i]);
        for (u32 j = i; j < L; j++) ora_ct_free(Cm[i * L + j]);
    }
    free(VR); free(VC); free(Cm);
    return st;
}

/* Multi-Ciphertext Sorting (section 5, Algorithm Multi-Ciphertext Sorting):
 * R_1..R_L = multi-ciphertext ranks of the blocks; for output block i and
 * source block j, M_{i,j} = Ind_0(ReplR(R_j) - (b(i-1)+1 || ... || b i)) with
 * Ind_0(x) = Cmp(x, -1/2) (1 - Cmp(x, 1/2)) on (x +- 1/2)/N (N = L b);
 * S_i = TransC(SumC(sum_j M_{i,j} * ReplR(B_j))).  Distinct inputs. */
int ora_sort_multi_depth(ora_cmp cm, ora_cmp ci) {
    /* multi rank, scaling, indicator, indicator product, M * V_R, SumC mask, TransC mask */
    return ora_rank_multi_depth(cm) + 5 + cmp_levels(ci);
}

int ora_sort_multi(const ora_keys *Kp, ora_ct *const *Bk, u32 L, u32 b, ora_cmp cm, ora_cmp ci,
                   ora_ct **S) {
    int st = check_N(Kp->P, b);
    if (st != ORA_OK) return st;
    if ((st = need_keys(Kp, b, 4)) != ORA_OK) return st;
    if (L < 1) return ORA_E_INVALID;
    for (u32 i = 0; i < L; i++)
        if (Bk[i]->level != Bk[0]->level) return ORA_E_INVALID;
    if (Bk[0]->level < ora_sort_multi_depth(cm, ci)) return ORA_E_DEPTH;
    const double dN = (double)L * (double)b;
    ora_ct **R = (ora_ct **)calloc(L, sizeof(ora_ct *));
    st = ora_rank_multi(Kp, Bk, L, b, cm, R);
    ora_ct **RR = (ora_ct **)calloc(L, sizeof(ora_ct *)), **VR = (ora_ct **)calloc(L, sizeof(ora_ct *));
    for (u32 j = 0; j < L; j++) {
        RR[j] = ora_repl_r(Kp, R[j], b, &st);
        VR[j] = ora_repl_r(Kp, Bk[j], b, &st);
    }
    double *steps = (double *)calloc((size_t)b * b, sizeof(double));
    for (u32 i = 0; i < L; i++) {
        for (u32 r = 0; r < b; r++)
            for (u32 c = 0; c < b; c++) steps[r * b + c] = -((double)b * i + r + 1);
        ora_ct *acc = NULL;
        for (u32 j = 0; j < L; j++) {
            ora_ct *X = ora_add_plain(RR[j], steps, b * b, &st);
            ora_ct *Xs = ora_cmul_to(X, ci.cheb > 0 ? 0.5 / dN : 1.0 / dN, X->level - 1, &st);
            if (ci.cheb > 0) replace(&Xs, plus_conj(Kp, Xs, &st));
            ora_ct *d1 = ora_add_const(Xs, 0.5 / dN);
            ora_ct *d2 = ora_add_const(Xs, -0.5 / dN);
            ora_ct *c1 = ora_cmp_sign(Kp, d1, ci, &st);
            ora_ct *c2 = ora_cmp_sign(Kp, d2, ci, &st);
            ora_ct *n2 = mul_int(c2, -1);
            ora_ct *o2 = ora_add_const(n2, 1.0);
            ora_ct *M = ora_mul(Kp, c1, o2, &st);
            ora_ct *VRa = ora_cmul_to(VR[j], 1.0, M->level, &st);
            ora_ct *P = ora_mul(Kp, M, VRa, &st);
            if (acc) replace(&acc, ora_add(acc, P)), ora_ct_free(P);
            else acc = P;
            ora_ct_free(X); ora_ct_free(Xs); ora_ct_free(d1); ora_ct_free(d2); ora_ct_free(c1); ora_ct_free(c2);
            ora_ct_free(n2); ora_ct_free(o2); ora_ct_free(M); ora_ct_free(VRa);
        }
        ora_ct *SC = ora_sum_c(Kp, acc, b, &st);
        S[i] = ora_trans_c(Kp, SC, b, &st);
        ora_ct_free(acc); ora_ct_free(SC);
    }
    free(steps);
    for (u32 j = 0; j < L; j++) { ora_ct_free(R[j]); ora_ct_free(RR[j]); ora_ct_free(VR[j]); }
    free(R); free(RR); free(VR);
    return st;
}

/* Galois elements needed by rank on N elements (left shifts as powers of 5) */
int ora_rank_galois(const ora_params *P, u32 Nr, u32 *out) {
    const u32 N = pow2_ceil(Nr); /* the padded layout */
    int cnt = 0, lg = ilog2(N);
    u64 h = P->n / 2;
    u64 shifts[256]; int ns = 0;
    for (int i = 1; i <= lg; i++) shifts[ns++] = h - (((u64)N * (N - 1)) >> i); /* TransR (right) */
    for (int i = 0; i < lg; i++) shifts[ns++] = h - ((u64)N << i);               /* ReplR (right) */
    for (int i = 0; i < lg; i++) shifts[ns++] = h - ((u64)1 << i);               /* ReplC (right) */
    for (int i = 0; i < lg; i++) shifts[ns++] = (u64)N << i;                     /* SumR (left) */
    for (int s = 0; s < ns; s++) {
        u32 g = gal_left(P, shifts[s] % h);
        int dup = 0;
        for (int k = 0; k < cnt; k++) if (out[k] == g) dup = 1;
        if (!dup) out[cnt++] = g;
    }
    return cnt;
}

u32 ora_galois_left(const ora_params *P, u64 k) { return gal_left(P, k); }

/* ------------------------------------------------------------------ */
/* Minimum with tie-correction (Order Statistic with k = 1, section    */
/* 3.2, plus the Tie-Correction Offset of section 4)                    */
/* ------------------------------------------------------------------ */
/* multiply by the signed integer K without rescaling (scale unchanged) */
ora_ct *ora_mul_int(const ora_ct *a, i64 K) { return mul_int(a, K); }

/* Order statistic k (Algorithm Order Statistic, section 3.2), optionally with
 * the tie-correction offset of section 4, generalised to a window of ranks
 * [a, b] (a = b = k is the order statistic).  Section 4 obtains the median of
 * an even count from the statistics N/2 and N/2 + 1 and a product by 1/2
 * after the inner product; with the window [N/2, N/2 + 1] both are extracted
 * by one mask, and value = SumC(O * V) / (b - a + 1) is the mean of the
 * statistics a..b, the factor folded into the plaintext constant that brings V
 * to the mask's level (no extra level; 1 when a = b).
 *
 * The indicator of "rank in [a, b]" is one-sided at the ends (a = 1:
 * Cmp(b + 1/2, k_j); b = N: Cmp(k_j, a - 1/2); the k_j are integral) and the
 * window Cmp(k_j, a - 1/2) (1 - Cmp(k_j, b + 1/2)) otherwise, every comparison
 * taken on its argument divided by N.  a = 1 with b = N selects everything and
 * is rejected.
 *
 * With tie-correction, k_j = SumR(C + E (delta_{j>=i} - 1/2)), E = C (4 - 4C)
 * (rank plus offset; their +1/2 and -1/2 cancel), which is a permutation of
 * 1..N: among equal values the lowest index is taken first.  N that is not a
 * power of two is padded (section 3.1) and needs tie-correction: the padding's
 * k_j are 0, outside every window with a >= 1, or selected by the a = 1 window
 * where V is zero; the one-hot keeps only the first N slots.
 * Without it, k_j is the rank R_j = SumR(C) + 1/2; the factor +-1/N is folded
 * into the comparator's last polynomial, and SumR keeps no row mask: the
 * other rows hold bounded garbage that O * V annihilates (V is zero outside
 * row 0).  onehot = MaskR(O, 0); value in slot 0. */
int ora_order_range_depth(u32 N, u32 a, u32 b, ora_cmp cm, ora_cmp ci, int tie) {
    int ind = cmp_levels(ci) + ((a > 1 && b < N) ? 1 : 0);
    /* [block mask,] TransR mask, comparator, [E, E*mask, SumR mask, scaling,] indicator, O*V, SumC mask;
     * without tie-correction a Chebyshev indicator keeps the SumR mask */
    return (pow2_ceil(N) != N ? 1 : 0) + 1 + cmp_levels(cm) + (tie ? 4 : 0) + ((!tie && ci.cheb > 0) ? 1 : 0) +
           ind + 2;
}

int ora_order_stat_depth(u32 N, u32 k, ora_cmp cm, ora_cmp ci, int tie) {
    return ora_order_range_depth(N, k, k, cm, ci, tie);
}

int ora_argmin_depth(ora_cmp cm, ora_cmp ci) { return ora_order_stat_depth(2, 1, cm, ci, 1); }

/* tie-corrected rank k_j = SumR(C + E (delta_{j>=i} - 1/2)), E = C (4 - 4C):
 * Rank plus the Tie-Correction Offset of section 4 (their +1/2 and -1/2
 * cancel), a permutation of 1..N.  Levels: TransR mask, comparator, E,
 * E * tie mask, SumR mask. */
static ora_ct *tie_rank(const ora_keys *Kp, const ora_ct *V, u32 Nr, ora_cmp cm, int *st) {
    const u32 N = pow2_ceil(Nr); /* layout; Nr < N pads (section 3.1) */
    ora_ct *C = ora_cmp_matrix(Kp, V, N, cm, st);
    if (N != Nr) replace(&C, block_mask(C, Nr, N, st));
    ora_ct *m4 = mul_int(C, -4);
    ora_ct *w = ora_add_const(m4, 4.0);
    ora_ct *E = ora_mul(Kp, C, w, st);
    double *tm = (double *)calloc((size_t)N * N, sizeof(double));
    for (u32 i = 0; i < N; i++)
        for (u32 j = 0; j < N; j++) tm[i * N + j] = j >= i ? 0.5 : -0.5;
    ora_ct *Et = ora_mul_plain(E, tm, N * N, st);
    free(tm);
    ora_ct *Ca = ora_cmul_to(C, 1.0, Et->level, st);
    ora_ct *X = ora_add(Ca, Et);
    ora_ct *kv = ora_sum_r(Kp, X, N, st);
    ora_ct_free(C); ora_ct_free(m4); ora_ct_free(w); ora_ct_free(E); ora_ct_free(Et); ora_ct_free(Ca);
    ora_ct_free(X);
    return kv;
}

ora_ct *ora_rank_tie(const ora_keys *Kp, const ora_ct *V, u32 N, ora_cmp cm, int *status) {
    int st = check_N_padded(Kp->P, N);
    if (st != ORA_OK) { *status = st; return NULL; }
    if ((st = need_keys(Kp, N, 1)) != ORA_OK) { *status = st; return NULL; }
    if (V->level < ora_rank_depth_n(N, cm, 1)) { *status = ORA_E_DEPTH; return NULL; }
    ora_ct *kv = tie_rank(Kp, V, N, cm, &st);
    *status = st;
    return kv;
}

static int order_range(const ora_keys *Kp, const ora_ct *V, u32 N, u32 a, u32 b, ora_cmp cm, ora_cmp ci,
                       int tie, ora_ct **onehot, ora_ct **value) {
    const u32 Np = pow2_ceil(N); /* the layout; N < Np pads */
    if (a < 1 || a > b || b > N || (a == 1 && b == N)) return ORA_E_INVALID;
    if (Np != N && !tie) return ORA_E_INVALID;
    if (V->level < ora_order_range_depth(N, a, b, cm, ci, tie)) return ORA_E_DEPTH;
    int st = ORA_OK;
    const double dN = (double)N, da = (double)a, db = (double)b;
    const int lower = a == 1; /* only the upper bound b + 1/2 is tested */
    /* a Chebyshev indicator takes the real part of its argument (plus_conj),
     * the 1/2 folded into the scaling; without tie-correction its argument
     * also keeps the SumR row mask, so that every slot lies in [-1, 1] */
    const int proj = ci.cheb > 0;
    const double sN = proj ? 2.0 * dN : dN;
    ora_ct *base; /* k_j (times -1/N when a = 1, else 1/N) */
    double off1, off2 = 0.0; /* constants giving the indicator argument(s) */
    if (tie) {
        ora_ct *kv = tie_rank(Kp, V, N, cm, &st);
        base = ora_cmul_to(kv, lower ? -1.0 / sN : 1.0 / sN, kv->level - 1, &st);
        if (lower) off1 = (db + 0.5) / dN;
        else off1 = (0.5 - da) / dN, off2 = (-0.5 - db) / dN;
        ora_ct_free(kv);
    } else {
        ora_ct *C = cmp_matrix_scaled(Kp, V, N, cm, lower ? -1.0 / sN : 1.0 / sN, &st);
        if (proj) {
            base = ora_sum_r(Kp, C, N, &st);
        } else {
            base = ct_copy(C);
            for (int i = 0; i < ilog2(N); i++) replace(&base, add_rot(Kp, base, (i64)N << i, &st));
        }
        /* SumR(C) = R_j - 1/2 */
        if (lower) off1 = db / dN;
        else off1 = (1.0 - da) / dN, off2 = -db / dN;
        ora_ct_free(C);
    }
    if (proj) replace(&base, plus_conj(Kp, base, &st));
    ora_ct *O;
    if (lower || b == N) {
        ora_ct *y = ora_add_const(base, off1);
        O = ora_cmp_sign(Kp, y, ci, &st);
        ora_ct_free(y);
    } else {
        ora_ct *d1 = ora_add_const(base, off1), *d2 = ora_add_const(base, off2);
        ora_ct *c1 = ora_cmp_sign(Kp, d1, ci, &st);
        ora_ct *c2 = ora_cmp_sign(Kp, d2, ci, &st);
        ora_ct *n2 = mul_int(c2, -1);
        ora_ct *o2 = ora_add_const(n2, 1.0);
        O = ora_mul(Kp, c1, o2, &st);
        ora_ct_free(d1); ora_ct_free(d2); ora_ct_free(c1); ora_ct_free(c2); ora_ct_free(n2); ora_ct_free(o2);
    }
    double *row = (double *)calloc(N, sizeof(double));
    for (u32 j = 0; j < N; j++) row[j] = 1.0;
    *onehot = ora_mul_plain(O, row, N, &st);
    free(row);
    ora_ct *Va = ora_cmul_to(V, 1.0 / (db - da + 1.0), O->level, &st);
    ora_ct *P = ora_mul(Kp, O, Va, &st);
    *value = ora_sum_c(Kp, P, Np, &st);
    ora_ct_free(base); ora_ct_free(O); ora_ct_free(Va); ora_ct_free(P);
    return st;
}

int ora_order_stat(const ora_keys *Kp, const ora_ct *V, u32 N, u32 k, ora_cmp cm, ora_cmp ci, int tie,
                   ora_ct **onehot, ora_ct **value) {
    int st = check_N(Kp->P, N);
    if (st != ORA_OK) return st;
    if ((st = need_keys(Kp, N, 2)) != ORA_OK) return st;
    if (k < 1 || k > N) return ORA_E_INVALID;
    return order_range(Kp, V, N, k, k, cm, ci, tie, onehot, value);
}

/* mean of the order statistics a..b (the median of an even N is a = N/2,
 * b = N/2 + 1; of an odd N, a = b = (N + 1)/2) */
int ora_order_range(const ora_keys *Kp, const ora_ct *V, u32 N, u32 a, u32 b, ora_cmp cm, ora_cmp ci, int tie,
                    ora_ct **onehot, ora_ct **value) {
    int st = check_N_padded(Kp->P, N);
    if (st != ORA_OK) return st;
    if ((st = need_keys(Kp, N, 2)) != ORA_OK) return st;
    return order_range(Kp, V, N, a, b, cm, ci, tie, onehot, value);
}

/* Order statistic with the value by division (section 3.2): without
 * tie-correction the mask O of the elements of rank k may hold several ones
 * (equal values share a rank) or none, and the value is
 * SumC(O * V) / SumC(O).  The division is Goldschmidt's: with the count
 * normalised to x = (2 / (N + 1)) SumC(MaskR(O)) in (0, 2),
 *   1/x ~ prod_{i<d} (1 + b^(2^i)),  b = 1 - x,
 * relative error b^(2^d), d >= 2; the first factor is affine, each later
 * one a squaring and a product.  value = ((2 / (N + 1)) SumC(O * V)) * prod.
 * If no element has rank k the numerator is zero (up to noise) and the
 * product at most 2^d.  Levels beyond the order statistic's (the count's
 * SumC mask runs beside the value's): the normalisation, d for the products
 * (the first also aligns a level), the final product -- d + 2. */
int ora_order_stat_div_depth(u32 N, u32 k, ora_cmp cm, ora_cmp ci, int iters) {
    return ora_order_stat_depth(N, k, cm, ci, 0) + iters + 2;
}

int ora_order_stat_div(const ora_keys *Kp, const ora_ct *V, u32 N, u32 k, ora_cmp cm, ora_cmp ci, int iters,
                       ora_ct **onehot, ora_ct **value) {
    if (iters < 2 || iters > 24) return ORA_E_INVALID;
    int st = check_N(Kp->P, N);
    if (st != ORA_OK) return st;
    if (k < 1 || k > N) return ORA_E_INVALID;
    if (V->level < ora_order_stat_div_depth(N, k, cm, ci, iters)) return ORA_E_DEPTH;
    ora_ct *num;
    st = ora_order_stat(Kp, V, N, k, cm, ci, 0, onehot, &num);
    if (st != ORA_OK) return st;
    const double s = 2.0 / ((double)N + 1.0);
    ora_ct *den = ora_sum_c(Kp, *onehot, N, &st);
    ora_ct *x = ora_cmul_to(den, s, den->level - 1, &st);
    ora_ct *nx = mul_int(x, -1);
    ora_ct *b = ora_add_const(nx, 1.0);   /* b = 1 - x */
    ora_ct *a = ora_add_const(nx, 2.0);   /* 1 + b */
    for (int i = 1; i < iters; i++) {
        replace(&b, ora_mul(Kp, b, b, &st));                 /* b^(2^i) */
        ora_ct *f = ora_add_const(b, 1.0);
        ora_ct *aa = align_to(a, f->level, &st);
        replace(&a, ora_mul(Kp, aa, f, &st));
        ora_ct_free(f); ora_ct_free(aa);
    }
    ora_ct *na = ora_cmul_to(num, s, a->level, &st);
    *value = ora_mul(Kp, na, a, &st);
    ora_ct_free(num); ora_ct_free(den); ora_ct_free(x); ora_ct_free(nx); ora_ct_free(b); ora_ct_free(a);
    ora_ct_free(na);
    return st;
}

/* the minimum with tie-correction: order statistic k = 1 */
int ora_argmin(const ora_keys *Kp, const ora_ct *V, u32 N, ora_cmp cm, ora_cmp ci, ora_ct **onehot,
               ora_ct **value) {
    return ora_order_stat(Kp, V, N, 1, cm, ci, 1, onehot, value);
}

/* ------------------------------------------------------------------ */
/* Sorting (Algorithm Sorting, section 3.3), distinct inputs            */
/* ------------------------------------------------------------------ */
/* levels: Rank, scaling, indicator, indicator product, M*V_R, SumC mask, TransC mask */
int ora_sort_depth(ora_cmp cm, ora_cmp ci) { return ora_rank_depth(cm) + 5 + cmp_levels(ci); }

/* R = Rank(V); R_R = ReplR(R); X = R_R - (1^N || ... || N^N);
 * M = Ind_0(X) = Cmp(X, -1/2) (1 - Cmp(X, 1/2)), the comparisons evaluated on
 * (X + 1/2)/N and (X - 1/2)/N; S = TransC(SumC(M * ReplR(V))). */
ora_ct *ora_sort(const ora_keys *Kp, const ora_ct *V, u32 N, ora_cmp cm, ora_cmp ci, int *status) {
    int st = check_N(Kp->P, N);
    if (st != ORA_OK) { *status = st; return NULL; }
    if ((st = need_keys(Kp, N, 4)) != ORA_OK) { *status = st; return NULL; }
    if (V->level < ora_sort_depth(cm, ci)) { *status = ORA_E_DEPTH; return NULL; }
    ora_ct *R = ora_rank(Kp, V, N, cm, &st);
    ora_ct *RR = ora_repl_r(Kp, R, N, &st);
    double *steps = (double *)calloc((size_t)N * N, sizeof(double));
    for (u32 i = 0; i < N; i++)
        for (u32 j = 0; j < N; j++) steps[i * N + j] = -(double)(i + 1);
    ora_ct *X = ora_add_plain(RR, steps, N * N, &st);
    free(steps);
    ora_ct *Xs = ora_cmul_to(X, ci.cheb > 0 ? 0.5 / (double)N : 1.0 / (double)N, X->level - 1, &st);
    if (ci.cheb > 0) replace(&Xs, plus_conj(Kp, Xs, &st));
    ora_ct *d1 = ora_add_const(Xs, 0.5 / (double)N);
    ora_ct *d2 = ora_add_const(Xs, -0.5 / (double)N);
    ora_ct *c1 = ora_cmp_sign(Kp, d1, ci, &st);
    ora_ct *c2 = ora_cmp_sign(Kp, d2, ci, &st);
    ora_ct *n2 = mul_int(c2, -1);
    ora_ct *o2 = ora_add_const(n2, 1.0);
    ora_ct *M = ora_mul(Kp, c1, o2, &st);
    ora_ct *VR = ora_repl_r(Kp, V, N, &st);
    ora_ct *VRa = ora_cmul_to(VR, 1.0, M->level, &st);
    ora_ct *P = ora_mul(Kp, M, VRa, &st);
    ora_ct *SC = ora_sum_c(Kp, P, N, &st);
    ora_ct *S = ora_trans_c(Kp, SC, N, &st);
    ora_ct_free(R); ora_ct_free(RR); ora_ct_free(X); ora_ct_free(Xs); ora_ct_free(d1); ora_ct_free(d2);
    ora_ct_free(c1); ora_ct_free(c2); ora_ct_free(n2); ora_ct_free(o2); ora_ct_free(M); ora_ct_free(VR);
    ora_ct_free(VRa); ora_ct_free(P); ora_ct_free(SC);
    *status = st;
    return S;
}

/* Column-form Sorting (section 3.3, the variant that saves the final
 * transposition): the comparator's operands are swapped and SumR becomes
 * SumC, so the ranks come out as a column, R'_i = SumC(Cmp(V_C, V_R)) + 1/2
 * at slot i N; the rest runs with rows and columns exchanged and
 * ReplC(TransR(V)) from the rank in place of ReplR(V):
 *   X = ReplC(R') - (1 || 2 || ... || N)^N  (column k holds k + 1),
 *   M = Ind_0(X) = Cmp(X, -1/2) (1 - Cmp(X, 1/2)) on (X +- 1/2)/N,
 *   S = SumR(M * ReplC(TransR(V))), the sorted vector in row 0.
 * Levels: TransR mask, comparator, SumC mask, scaling, indicator, indicator
 * product, M * V_C, SumR mask. */
int ora_sort_col_depth(ora_cmp cm, ora_cmp ci) { return ora_rank_depth(cm) + 4 + cmp_levels(ci); }

ora_ct *ora_sort_col(const ora_keys *Kp, const ora_ct *V, u32 N, ora_cmp cm, ora_cmp ci, int *status) {
    int st = check_N(Kp->P, N);
    if (st != ORA_OK) { *status = st; return NULL; }
    if ((st = need_keys(Kp, N, 2)) != ORA_OK) { *status = st; return NULL; }
    if (!cmp_valid(cm) || !cmp_valid(ci)) { *status = ORA_E_INVALID; return NULL; }
    if (V->level < ora_sort_col_depth(cm, ci)) { *status = ORA_E_DEPTH; return NULL; }
    const double dN = (double)N;
    ora_ct *VR = ora_repl_r(Kp, V, N, &st);
    ora_ct *T = ora_trans_r(Kp, V, N, &st);
    ora_ct *VC = ora_repl_c(Kp, T, N, &st);
    ora_ct *VRa = ora_cmul_to(VR, 1.0, VC->level, &st);
    ora_ct *D = ora_sub(VC, VRa);
    ora_ct *C = cmp_sign_scaled(Kp, D, cm, 1.0, &st);
    ora_ct *SC = ora_sum_c(Kp, C, N, &st);
    double *z = (double *)calloc((size_t)N * N, sizeof(double));
    for (u32 i = 0; i < N; i++) z[(size_t)i * N] = 0.5;
    ora_ct *R = ora_add_plain(SC, z, N * N, &st);
    ora_ct *RC = ora_repl_c(Kp, R, N, &st);
    for (u32 i = 0; i < N; i++)
        for (u32 k = 0; k < N; k++) z[(size_t)i * N + k] = -(double)(k + 1);
    ora_ct *X = ora_add_plain(RC, z, N * N, &st);
    free(z);
    ora_ct *Xs = ora_cmul_to(X, ci.cheb > 0 ? 0.5 / dN : 1.0 / dN, X->level - 1, &st);
    if (ci.cheb > 0) replace(&Xs, plus_conj(Kp, Xs, &st));
    ora_ct *d1 = ora_add_const(Xs, 0.5 / dN);
    ora_ct *d2 = ora_add_const(Xs, -0.5 / dN);
    ora_ct *c1 = ora_cmp_sign(Kp, d1, ci, &st);
    ora_ct *c2 = ora_cmp_sign(Kp, d2, ci, &st);
    ora_ct *n2 = mul_int(c2, -1);
    ora_ct *o2 = ora_add_const(n2, 1.0);
    ora_ct *M = ora_mul(Kp, c1, o2, &st);
    ora_ct *VCa = ora_cmul_to(VC, 1.0, M->level, &st);
    ora_ct *P = ora_mul(Kp, M, VCa, &st);
    ora_ct *S = ora_sum_r(Kp, P, N, &st);
    ora_ct_free(VR); ora_ct_free(T); ora_ct_free(VC); ora_ct_free(VRa); ora_ct_free(D); ora_ct_free(C);
    ora_ct_free(SC); ora_ct_free(R); ora_ct_free(RC); ora_ct_free(X); ora_ct_free(Xs); ora_ct_free(d1);
    ora_ct_free(d2); ora_ct_free(c1); ora_ct_free(c2); ora_ct_free(n2); ora_ct_free(o2); ora_ct_free(M);
    ora_ct_free(VCa); ora_ct_free(P);
    *status = st;
    return S;
}

/* Galois elements needed by the circuits: bit 0 rank, bit 1 argmin (adds
 * SumC), bit 2 sort (adds SumC and TransC) */
int ora_circuit_galois(const ora_params *P, u32 Nr, int what, u32 *out) {
    const u32 N = pow2_ceil(Nr);
    int cnt = ora_rank_galois(P, N, out), lg = ilog2(N);
    u64 h = P->n / 2;
    u64 shifts[64]; int ns = 0;
    if (what & 6)
        for (int i = 0; i < lg; i++) shifts[ns++] = (u64)1 << i;                  /* SumC (left) */
    if (what & 4)
        for (int i = 1; i <= lg; i++) shifts[ns++] = ((u64)N * (N - 1)) >> i;     /* TransC (left) */
    for (int s = 0; s < ns; s++) {
        u32 g = gal_left(P, shifts[s] % h);
        int dup = 0;
        for (int k = 0; k < cnt; k++) if (out[k] == g) dup = 1;
        if (!dup) out[cnt++] = g;
    }
    if (what & 6) out[cnt++] = (u32)(2 * P->n - 1); /* conjugation: real part of a Chebyshev indicator's argument */
    return cnt;
}
