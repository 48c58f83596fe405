// host_math.h -- host-side number theory, parameter derivation, ChaCha20
// sampling and the slot encoder of the ckr library.
#pragma once
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace ckr {

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;

struct Error {
    int status;
    std::string msg;
};

// ---- modular helpers (host) ----
u64 hmul(u64 a, u64 b, u64 m);
u64 hpow(u64 a, u64 e, u64 m);
u64 hinv(u64 a, u64 m);  // m prime
u64 hred(i64 v, u64 m);
bool hprime(u64 n);

// ---- parameter set ----
struct Params {
    int logn = 0;
    u64 n = 0;
    int L = 0, nq = 0, K = 0, dnum = 0, alpha = 0, log_scale = 0;
    std::vector<u64> mod;      // q_0..q_L then p_0..p_{K-1}
    std::vector<u64> psi;      // primitive 2n-th root per modulus
    std::vector<double> scale; // D_l, l = 0..L
    int nmod() const { return nq + K; }
    // digit j of the chain covers q indices [j*alpha, min((j+1)*alpha, nq))
    int beta(int level) const { return (level + 1 + alpha - 1) / alpha; }
};
// builds the chain; throws Error on bad input
Params make_params(int logn, int nq, int q0_bits, int log_scale, int K, int p_bits, int dnum);

// ---- ChaCha20 (RFC 8439) streams ----
void chacha20_block(const uint8_t key[32], u32 counter, const uint8_t nonce[12], u32 out[16]);
class Stream {
  public:
    Stream(const uint8_t key[32], u32 purpose, u64 id);
    u32 next32();
    u64 next64();
    int ternary();
    int cbd21();
    u64 uniform(u64 q);

  private:
    uint8_t key_[32], nonce_[12];
    u32 ctr_ = 0, buf_[16];
    int pos_ = 16;
};
enum Purpose : u32 {
    kSecret = 1, kPkA = 2, kPkE = 3, kKsA = 4, kKsE = 5, kEncU = 6, kEncE0 = 7, kEncE1 = 8
};

// ---- slot encoding (binary128) ----
// m_j = round_half_away((2 D / n) Re(sum_k z_k zeta^{-j 5^k})), zeta = exp(i pi / n)
// returns false if a coefficient exceeds 2^62
bool encode_slots(int logn, const double *z, u32 count, double scale, i64 *m);
// real parts of slots [0, count) of the polynomial m / scale
void decode_slots(int logn, const i64 *m, double scale, u32 count, double *z);

// ---- Chebyshev interpolant of the comparison function (binary128) ----
// c[0 .. 2^(D-1)): coefficients of the degree 2^(D-1) - 1 interpolant, at the
// 2^(D-1) Chebyshev nodes of [-1, 1], of the function that is 1 for d > 0
// and 0 for d < 0
void cheb_step_coeffs(int D, double *c);

}  // namespace ckr
