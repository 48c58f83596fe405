// host_math.cpp -- number theory, parameter derivation, ChaCha20 sampling and
// the binary128 slot encoder of the ckr library (host only).
#include "host_math.h"

#include <quadmath.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

namespace ckr {

typedef unsigned __int128 u128;

u64 hmul(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
u64 hpow(u64 a, u64 e, u64 m) {
    u64 r = 1 % m;
    a %= m;
    for (; e; e >>= 1) {
        if (e & 1) r = hmul(r, a, m);
        a = hmul(a, a, m);
    }
    return r;
}
u64 hinv(u64 a, u64 m) { return hpow(a % m, m - 2, m); }
u64 hred(i64 v, u64 m) {
    i64 r = v % (i64)m;
    return (u64)(r < 0 ? r + (i64)m : r);
}

// Miller-Rabin with the seven bases known to be deterministic for all 64-bit n
bool hprime(u64 n) {
    if (n < 2) return false;
    for (u64 p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
        if (n % p == 0) return n == p;
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) d >>= 1, s++;
    for (u64 a : {2ull, 325ull, 9375ull, 28178ull, 450775ull, 9780504ull, 1795265022ull}) {
        u64 x = hpow(a % n, d, n);
        if (x == 0 || x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s && comp; r++) {
            x = hmul(x, x, n);
            if (x == n - 1) comp = false;
        }
        if (comp) return false;
    }
    return true;
}

static bool contains(const std::vector<u64> &v, u64 x) {
    for (u64 y : v)
        if (y == x) return true;
    return false;
}

Params make_params(int logn, int nq, int q0_bits, int log_scale, int K, int p_bits, int dnum) {
    if (logn < 10 || logn > 17) throw Error{-1, "log_n must be in [10, 17]"};
    if (nq < 1 || K < 1 || nq + K > 128 || dnum < 1 || dnum > nq) throw Error{-1, "bad prime counts"};
    if (q0_bits < 20 || q0_bits > 50 || p_bits < 20 || p_bits > 50 || log_scale < 20 || log_scale > 48)
        throw Error{-1, "prime sizes must stay below 2^50"};
    Params P;
    P.logn = logn;
    P.n = 1ull << logn;
    P.nq = nq;
    P.L = nq - 1;
    P.K = K;
    P.dnum = dnum;
    P.alpha = (nq + dnum - 1) / dnum;
    P.log_scale = log_scale;
    const u64 step = 2 * P.n;
    std::vector<u64> used;
    auto top_prime = [&](int bits) {
        u64 c = ((1ull << bits) - 1) / step * step + 1;
        while (!(hprime(c) && !contains(used, c))) c -= step;
        return c;
    };
    std::vector<u64> sp;
    for (int k = 0; k < K; k++) {
        u64 p = top_prime(p_bits);
        used.push_back(p);
        sp.push_back(p);
    }
    P.mod.assign(nq + K, 0);
    P.scale.assign(nq, 0.0);
    P.mod[0] = top_prime(q0_bits);
    used.push_back(P.mod[0]);
    P.scale[P.L] = std::ldexp(1.0, log_scale);
    for (int l = P.L; l >= 1; l--) {
        const double D = P.scale[l];
        // candidates 1 mod 2n on both sides of D, nearest first; ties go to the lower one
        u64 below = (u64)std::floor(D);
        below -= (below - 1) % step;
        u64 above = below + step;
        u64 pick = 0;
        while (!pick) {
            if (D - (double)below <= (double)above - D) {
                if (hprime(below) && !contains(used, below)) pick = below;
                below -= step;
            } else {
                if (hprime(above) && !contains(used, above)) pick = above;
                above += step;
            }
        }
        used.push_back(pick);
        P.mod[l] = pick;
        P.scale[l - 1] = (D * D) / (double)pick;
    }
    for (int k = 0; k < K; k++) P.mod[nq + k] = sp[k];
    // any primitive 2n-th root works: results are defined in the coefficient domain
    P.psi.resize(nq + K);
    for (int t = 0; t < nq + K; t++) {
        const u64 q = P.mod[t];
        for (u64 x = 3;; x += 2) {
            u64 w = hpow(x, (q - 1) / step, q);
            if (hpow(w, P.n, q) == q - 1) {
                P.psi[t] = w;
                break;
            }
        }
    }
    return P;
}

// ---------------------------------------------------------------- ChaCha20
static inline u32 rl(u32 v, int c) { return (v << c) | (v >> (32 - c)); }
static inline void quarter(u32 &a, u32 &b, u32 &c, u32 &d) {
    a += b; d = rl(d ^ a, 16);
    c += d; b = rl(b ^ c, 12);
    a += b; d = rl(d ^ a, 8);
    c += d; b = rl(b ^ c, 7);
}
static inline u32 le32(const uint8_t *p) { return p[0] | (p[1] << 8) | (p[2] << 16) | ((u32)p[3] << 24); }

void chacha20_block(const uint8_t key[32], u32 counter, const uint8_t nonce[12], u32 out[16]) {
    u32 init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
    for (int i = 0; i < 8; i++) init[4 + i] = le32(key + 4 * i);
    init[12] = counter;
    for (int i = 0; i < 3; i++) init[13 + i] = le32(nonce + 4 * i);
    u32 w[16];
    std::memcpy(w, init, sizeof w);
    for (int round = 0; round < 20; round += 2) {
        quarter(w[0], w[4], w[8], w[12]);
        quarter(w[1], w[5], w[9], w[13]);
        quarter(w[2], w[6], w[10], w[14]);
        quarter(w[3], w[7], w[11], w[15]);
        quarter(w[0], w[5], w[10], w[15]);
        quarter(w[1], w[6], w[11], w[12]);
        quarter(w[2], w[7], w[8], w[13]);
        quarter(w[3], w[4], w[9], w[14]);
    }
    for (int i = 0; i < 16; i++) out[i] = w[i] + init[i];
}

Stream::Stream(const uint8_t key[32], u32 purpose, u64 id) {
    std::memcpy(key_, key, 32);
    for (int i = 0; i < 4; i++) nonce_[i] = (uint8_t)(purpose >> (8 * i));
    for (int i = 0; i < 8; i++) nonce_[4 + i] = (uint8_t)(id >> (8 * i));
}
u32 Stream::next32() {
    if (pos_ == 16) {
        chacha20_block(key_, ctr_++, nonce_, buf_);
        pos_ = 0;
    }
    return buf_[pos_++];
}
u64 Stream::next64() {
    u64 lo = next32();
    return lo | ((u64)next32() << 32);
}
int Stream::ternary() {
    for (;;) {
        u32 v = next32() & 3u;
        if (v != 3u) return (int)v - 1;
    }
}
int Stream::cbd21() {
    u64 w = next64();
    return __builtin_popcountll(w & 0x1FFFFFull) - __builtin_popcountll((w >> 21) & 0x1FFFFFull);
}
u64 Stream::uniform(u64 q) {
    const int bits = 64 - __builtin_clzll(q);
    const u64 mask = bits == 64 ? ~0ull : ((1ull << bits) - 1);
    for (;;) {
        u64 v = next64() & mask;
        if (v < q) return v;
    }
}

// ---------------------------------------------------------------- encoder
// With g_k = 5^k mod 2n = 2 h_k + 1 and omega = zeta^2,
//   sum_k z_k zeta^{-j g_k} = zeta^{-j} * sum_h b_h omega^{-j h},  b_{h_k} = z_k,
// so encoding is one length-n DFT (radix-2 decimation in frequency, binary128)
// followed by a twist.
typedef __complex128 cq;

struct FftTables {
    std::vector<cq> root;   // omega^{-k}, k < n/2
    std::vector<cq> twist;  // zeta^{-j}, j < n
    std::vector<u32> h;     // h_k, k < n/2
};

static const FftTables &tables(int logn) {
    static std::mutex mu;
    static std::map<int, FftTables> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(logn);
    if (it != cache.end()) return it->second;
    FftTables T;
    const u64 n = 1ull << logn;
    T.root.resize(n / 2);
    for (u64 k = 0; k < n / 2; k++) {
        __float128 a = 2 * M_PIq * (__float128)k / (__float128)n;
        __real__ T.root[k] = cosq(a);
        __imag__ T.root[k] = -sinq(a);
    }
    T.twist.resize(n);
    for (u64 j = 0; j < n; j++) {
        __float128 a = M_PIq * (__float128)j / (__float128)n;
        __real__ T.twist[j] = cosq(a);
        __imag__ T.twist[j] = -sinq(a);
    }
    T.h.resize(n / 2);
    u64 g = 1;
    for (u64 k = 0; k < n / 2; k++) {
        T.h[k] = (u32)((g - 1) / 2);
        g = (g * 5) % (2 * n);
    }
    return cache.emplace(logn, std::move(T)).first->second;
}

static u64 brev_bits(u64 x, int bits) {
    u64 r = 0;
    for (int i = 0; i < bits; i++) r |= ((x >> i) & 1) << (bits - 1 - i);
    return r;
}

// in-place DIF: natural-order input, output X[brev(j)] = sum_h x_h omega^{-j h}
// (conj = true uses omega^{+j h})
static void dif(std::vector<cq> &x, int logn, const FftTables &T, bool conj) {
    const u64 n = 1ull << logn;
    for (u64 half = n / 2, stride = 1; half >= 1; half >>= 1, stride <<= 1) {
        for (u64 blk = 0; blk < n; blk += 2 * half)
            for (u64 j = 0; j < half; j++) {
                cq w = T.root[j * stride];
                if (conj) __imag__ w = -__imag__ w;
                cq a = x[blk + j], b = x[blk + j + half];
                x[blk + j] = a + b;
                x[blk + j + half] = (a - b) * w;
            }
    }
}

// With n = 2^(D-1) nodes x_j = cos(pi (j + 1/2) / n), the interpolation
// coefficient is c_k = (2/n) sum_{x_j > 0} cos(k pi (j + 1/2) / n) (halved for
// k = 0); the positive nodes are j < n/2, and the cosine sum over them is
// sin(k pi / 2) / (2 sin(k pi / 2n)): zero for even k > 0, and for odd k
// c_k = (-1)^((k-1)/2) / (n sin(k pi / 2n)).
void cheb_step_coeffs(int D, double *c) {
    const long n = 1L << (D - 1);
    c[0] = 0.5;
    for (long k = 1; k < n; k++) {
        if (k % 2 == 0) {
            c[k] = 0.0;
            continue;
        }
        const __float128 s = sinq(M_PIq * (__float128)k / (__float128)(2 * n));
        const __float128 sign = ((k - 1) / 2) % 2 ? -1 : 1;
        c[k] = (double)(sign / ((__float128)n * s));
    }
}

bool encode_slots(int logn, const double *z, u32 count, double scale, i64 *m) {
    const FftTables &T = tables(logn);
    const u64 n = 1ull << logn;
    std::vector<cq> b(n, 0);
    for (u32 k = 0; k < count; k++) __real__ b[T.h[k]] = (__float128)z[k];
    dif(b, logn, T, false);
    const __float128 f = 2 * (__float128)scale / (__float128)n;
    bool ok = true;
    for (u64 j = 0; j < n; j++) {
        cq a = b[brev_bits(j, logn)] * T.twist[j];
        __float128 v = f * crealq(a);
        __float128 r = v < 0 ? -floorq(0.5Q - v) : floorq(v + 0.5Q);
        if (fabsq(r) > 0x1p62Q) {
            ok = false;
            r = 0;
        }
        m[j] = (i64)r;
    }
    return ok;
}

void decode_slots(int logn, const i64 *m, double scale, u32 count, double *z) {
    const FftTables &T = tables(logn);
    const u64 n = 1ull << logn;
    std::vector<cq> c(n);
    for (u64 j = 0; j < n; j++) {
        cq tw = T.twist[j];
        __imag__ tw = -__imag__ tw;  // zeta^{+j}
        c[j] = (__float128)m[j] * tw;
    }
    dif(c, logn, T, true);
    for (u32 k = 0; k < count; k++) z[k] = (double)(crealq(c[brev_bits(T.h[k], logn)]) / (__float128)scale);
}

}  // namespace ckr
