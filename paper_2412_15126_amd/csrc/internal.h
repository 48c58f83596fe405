// internal.h -- declarations shared by the host code and the HIP kernels of
// the ckr library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

namespace ckr {

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;

constexpr int kMaxMod = 128;   // moduli (q chain + special primes)
constexpr int kMaxLimbArgs = 64;

// limb t of a batch of limbs is reduced modulo  t < split ? t + off0 : t - split + off1
struct LimbMap {
    int split, off0, off1;
    __host__ __device__ int operator()(int t) const { return t < split ? t + off0 : t - split + off1; }
};
inline LimbMap plain_map(int first = 0) { return LimbMap{1 << 30, first, 0}; }

// per-limb scalar operand passed by value: value and value/q as doubles
struct LimbScalars {
    double v[kMaxLimbArgs];
    double vq[kMaxLimbArgs];
};

// device-resident tables for one ring
struct DevTables {
    int logn;
    int nmod;
    double2 *mq;      // [nmod] {q, 1/q}
    u64 *qi;          // [nmod] q as integers
    double2 *tw_last; // [nmod][2]: {n^-1, n^-1/q}, {psi^{-brev(1)} n^-1, ./q}
    double *twq_fwd;  // [nmod][n] w/q, w = psi^{brev(i)} (the passes recover w = rint(w/q * q))
    double *twq_inv;  // [nmod][n] w/q, w = psi^{-brev(i)}
    int ntt_variant[2][2] = {{0, 0}, {0, 0}};  // [inverse][pass]: tile variant chosen by the autotuner
    int row_ip_variant = 7;                      // tile of the fused row pass + inner product
};
constexpr int kNttVariants = 5;
constexpr int kRowIpVariants = 8;

// description of a batch of limbs: `polys` groups of `limbs` limbs, group p
// starting at base + p * poly_stride, limbs n words apart
struct LimbBatch {
    u64 *base;
    int limbs;
    int polys;
    size_t poly_stride;
    LimbMap map;
    const u64 *src = nullptr;  // when set, the first pass reads limb t of poly p from src + p*src_stride + t*n
    size_t src_stride = 0;
    u32 gal = 0;  // when > 1, the first pass reads its input through the automorphism sigma_gal (src must be set)
};

// ---- kernels (ckr_kernels.hip) ------------------------------------------
void k_ntt(const DevTables &T, const LimbBatch &b, bool inverse, hipStream_t s);
// one pass of the two-pass transform: pass 0 runs first (columns forward, rows inverse)
void k_ntt_pass(const DevTables &T, const LimbBatch &b, bool inverse, int pass, hipStream_t s);
// the same pass with an explicit tile variant (autotuning); variant < kNttVariants
void k_ntt_pass_variant(const DevTables &T, const LimbBatch &b, bool inverse, int pass, int variant, hipStream_t s);

// optional fused prologue / epilogue of the forward transform.
// prologue (first pass): limb t of poly p is read from src + p*src_stride (one
//   limb per poly) and reduced modulo the limb's own prime.
// epilogue (last pass): instead of storing y, poly p = 2b + k stores
//   out = (x - y) * c[t] (+ add when bit k of add_mask is set), where each of
//   out, x, add addresses poly p at base + b*stride + k*off.
struct NttFuse {
    bool pro = false, epi = false;
    const u64 *src = nullptr;
    size_t src_stride = 0;
    u64 *out = nullptr;
    size_t out_stride = 0, out_off = 0;
    const u64 *x = nullptr;
    size_t x_stride = 0, x_off = 0;
    const u64 *add = nullptr;
    size_t add_stride = 0, add_off = 0;
    int add_mask = 0;
    u32 add_gal = 0;            // when > 1, add is read through the automorphism sigma_add_gal
    const u64 *add2 = nullptr;  // a second addend, addressed like add
    size_t add2_stride = 0, add2_off = 0;
    int add2_mask = 0;
    LimbScalars c;
    double pro_q = 0.0;  // prologue: when > 0, the input limb's residues mod pro_q are taken in (-pro_q/2, pro_q/2)
    // fused ModDown + rescale: the prologue adds limb t of src2 (poly p at
    // src2 + p*src2_stride) times c2[t] to the broadcast limb, and the
    // epilogue (pre) takes (x*c2[t] + add - y) * c[t] instead of (x - y) * c[t] + add
    const u64 *src2 = nullptr;
    size_t src2_stride = 0;
    bool pre = false;
    LimbScalars c2;
    // epilogue: x taken slot-wise times the plaintext limb xmul + t*n (the
    // same for every poly) before the combine; add2 subtracted, not added
    const u64 *xmul = nullptr;
    bool add2_sub = false;
};
void k_ntt_fused(const DevTables &T, const LimbBatch &b, const NttFuse &f, int pass, hipStream_t s);

// out = a + b, a - b (mod q) over a batch of limbs (same geometry for all three)
void k_add(const DevTables &T, u64 *out, const u64 *a, const u64 *b, int limbs, int polys, size_t stride_o,
           size_t stride_a, size_t stride_b, LimbMap map, bool sub, hipStream_t s);
// limb t of each of `polys` polynomials (stride apart) += c[t]
void k_add_scalar(const DevTables &T, u64 *data, int limbs, int polys, size_t stride, LimbMap map,
                  const LimbScalars &c, hipStream_t s);
// out[p][t] = a[p][t] * c[t]
void k_mul_scalar(const DevTables &T, u64 *out, const u64 *a, int limbs, int polys, size_t stride_o, size_t stride_a,
                  LimbMap map, const LimbScalars &c, hipStream_t s);
// Linear combinations with integer constants of nt ciphertext batches of one
// level (limbs q_0 .. q_{limbs-1}), B entries each:
//   out[o][b] = sum_i K[o][i] * term[i][b]   (mod q_t, every limb t),
// out laid out [nout][B][2][limbs][n].  K is given per limb as
// k[(o * nt + i) * limbs + t] = (K mod q_t, (K mod q_t) / q_t).
constexpr int kMaxLinTerms = 64;
struct LinComb {
    const u64 *term[kMaxLinTerms];
    u64 *out = nullptr;
    const double2 *k = nullptr;
    int nt = 0, nout = 0, limbs = 0, B = 0;
};
void k_lincomb(const DevTables &T, const LinComb &a, hipStream_t s);
// out[p][t] = a[p][t] (*|+) pt[t]
void k_mul_pt(const DevTables &T, u64 *out, const u64 *a, const u64 *pt, int limbs, int polys, size_t stride_o,
              size_t stride_a, LimbMap map, bool add, hipStream_t s);
// per batch entry b: d = [d0 d1 d2] at d + b*sd (polys (limbs*n) apart), a = [a0 a1] at a + b*sa,
// b = [b0 b1] at bb + b*sb;  d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1
void k_tensor(const DevTables &T, u64 *d, const u64 *a, const u64 *bb, int limbs, int batch, size_t sd, size_t sa,
              size_t sb, hipStream_t s);
// evaluation-domain automorphism sigma_g on `polys` x `limbs` limbs
void k_automorph(const DevTables &T, u64 *out, const u64 *in, int limbs, int polys, size_t stride_o, size_t stride_i,
                 u32 g, hipStream_t s);

// fast base conversion (coefficient domain): src limbs src[0..ns) with moduli
// src_mod[i]; targets limbs out + j*n, moduli tgt_mod[j]; tables hinv[ns] and
// hmod[ns][nt] ({v, v/m} pairs) in device memory
constexpr int kMaxBConvSrc = 16;
struct BConvTab {
    int ns, nt;
    int src_mod[kMaxBConvSrc];
    int tgt_mod[kMaxLimbArgs];
    int tgt_slot[kMaxLimbArgs];  // output limb index of target j
    double2 *hinv;  // [ns]
    double2 *hmod;  // [ns][nt]
    // rounding ModDown (null otherwise): pre[i] = h mod p_i is added to source
    // i's residue and post[j] = h mod t_j subtracted from target j,
    // h = (P - 1)/2: the conversion of X + h, minus h.  The conversion is
    // then exact: its overflow u = floor(sum_i y_i * rinv[i]) (IEEE double,
    // in source order, no fused operations) times pmod[j] = P mod t_j is
    // subtracted as well, so target j receives [(X + h) mod P - h]_{t_j}.
    double *pre;    // [ns]
    double *post;   // [nt]
    double *rinv;   // [ns] 1/p_i
    double2 *pmod;  // [nt] {P mod t_j, (P mod t_j) / t_j}
};
void k_bconv(const DevTables &T, u64 *out, const u64 *src, const BConvTab &tab, int batch, size_t stride_o,
             size_t stride_i, hipStream_t s);


// key-switch inner product over E limbs (eval domain):
//   accb[t] = sum_j X_j[t] * kb_j[t], acca[t] = sum_j X_j[t] * ka_j[t]
// X_j[t] = d[t] if limb t (t <= level) lies in digit j, else ext[j][t]
struct IPArgs {
    const u64 *d;        // [level+1][n]
    const u64 *ext;      // [beta][E][n]
    const u64 *key;      // [beta_key][2][Ek][n]
    u64 *accb, *acca;    // [E][n]
    int level, E, beta, alpha, Ek, lmax_key, nq;
    int B;                       // batch of inputs sharing the key
    size_t sd, sext, sacc;       // batch strides of d, ext, accb/acca
    u32 gal = 0;                 // when > 1, d is read through the automorphism sigma_gal
    bool inv_p = false;          // limbs t > level (special primes): store them after the inverse
                                 // transform's row pass (ModDown's first pass), lazily reduced
};
// computed with the forward row pass of ext fused in front: ext holds the
// extended limbs after their column pass only
void k_ntt_row_ip(const DevTables &T, const IPArgs &a, hipStream_t s);

// reduce arbitrary uint64 values to canonical residues (import check helper):
// flags[0] set to 1 if any value >= its modulus
void k_check_range(const DevTables &T, const u64 *data, int limbs, int polys, size_t stride, int *flag, hipStream_t s);

}  // namespace ckr
