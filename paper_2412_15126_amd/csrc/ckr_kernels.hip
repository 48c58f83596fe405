// ckr_kernels.hip -- gfx950 kernels of the RNS-CKKS path.
//
// Residues live in HBM as canonical uint64 in [0, q), q < 2^50, limb-major
// (each limb = n contiguous words).  Inside a kernel they are carried as
// doubles: every value below 2^52 is an exact double, so a modular product
// is computed exactly with FP64 FMAs (error-free product split plus a
// rounded quotient estimate), which runs at the full FP64 vector rate on
// CDNA4 -- faster than 64-bit integer multiplies.  No MFMA: the work is
// exact modular integer arithmetic.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace ckr {

#define C52 4503599627370496.0  // 2^52
#define C53 9007199254740992.0  // 2^53

// ------------------------------------------------------------------------
// exact modular arithmetic in FP64
// ------------------------------------------------------------------------
// uint64 x < 2^52  ->  double (exact)
__device__ __forceinline__ double u2d(u64 x) {
    return __hiloint2double(0x43300000 | (int)(x >> 32), (int)(u32)x) - C52;
}
// integer-valued double in [0, 2^52)  ->  uint64
__device__ __forceinline__ u64 d2u(double d) {
    return (u64)__double_as_longlong(d + C52) & 0xFFFFFFFFFFFFFull;
}

// x * w mod q for a constant w with wq = w/q; x in [0, 2^52).
// The product is split exactly (hi + lo), the quotient estimate round(x*wq)
// is within 1 of x*w/q, so the result lands in (0, 2q).
__device__ __forceinline__ double mm_lazy(double x, double w, double wq, double q) {
    double hi = x * w;
    double lo = __fma_rn(x, w, -hi);
    double k = __fma_rn(x, wq, C52) - (C52 + 1.0);
    return __fma_rn(-k, q, hi) + lo;
}
// x * y mod q for canonical x, y < q < 2^50: result in (-0.75q, 0.75q)
__device__ __forceinline__ double mm_signed(double x, double y, double q, double qinv) {
    double hi = x * y;
    double lo = __fma_rn(x, y, -hi);
    double k = __fma_rn(hi, qinv, C52) - C52;
    return __fma_rn(-k, q, hi) + lo;
}
__device__ __forceinline__ double red1(double x, double q) { return x >= q ? x - q : x; }  // [0,2q) -> [0,q)
__device__ __forceinline__ double pos1(double x, double q) { return x < 0 ? x + q : x; }   // (-q,q) -> [0,q)
// integer-valued x in (-2^53, 2^53) -> x mod q in [0, q), qinv = fl(1/q).
// k = rint(x qinv) is within 1/2 + 2/q of x/q, so x - k q is an integer in
// (-q, q): the FMA forms it exactly and one correction makes it canonical.
__device__ __forceinline__ double red_any(double x, double q, double qinv) {
    const double r = __fma_rn(-rint(x * qinv), q, x);
    return r < 0 ? r + q : r;
}

// one 64-bit value through a DPP quad permutation (CTRL: the quad_perm selector)
template <int CTRL>
__device__ __forceinline__ double qperm(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
// 4 x 4 transpose inside each quad of lanes (lane l's x[j] <- lane j's x[l]):
// swap the off-diagonal 2 x 2 blocks across lanes l ^ 2, then the
// off-diagonal entries of each block across lanes l ^ 1
__device__ __forceinline__ void quad_transpose(double *x) {
    const int l = threadIdx.x & 3;
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const double recv = qperm<0x4E>((l & 2) ? x[j] : x[j + 2]);  // quad_perm [2,3,0,1]
        if (l & 2) x[j] = recv;
        else x[j + 2] = recv;
    }
#pragma unroll
    for (int j = 0; j < 4; j += 2) {
        const double recv = qperm<0xB1>((l & 1) ? x[j] : x[j + 1]);  // quad_perm [1,0,3,2]
        if (l & 1) x[j] = recv;
        else x[j + 1] = recv;
    }
}

// Evaluation-domain automorphism sigma_g: position i holds a(psi^{2 brev(i) + 1}),
// and sigma_g(a) at i is a at the position of exponent (2 brev(i) + 1) g.  The
// map keeps aligned blocks of 2^k positions together (for every k), so
// gathers through it stay coalesced.
__device__ __forceinline__ u32 gal_src(u32 i, int logn, u32 g) {
    const u32 e = (u32)((((u64)(__brev(i) >> (32 - logn)) * 2 + 1) * g) & ((2u << logn) - 1));
    return __brev((e - 1) >> 1) >> (32 - logn);
}

// ------------------------------------------------------------------------
// negacyclic NTT: one pass of a two-pass decomposition n = n1 * n2
// ------------------------------------------------------------------------
// Forward transform (Cooley-Tukey, merged psi twiddles): stage g pairs indices
// j, j + n/2^{g+1} with twiddle w[2^g + (j >> (logn - g))].  The first logn1
// stages act on columns {c + n2 r}, the rest on contiguous rows of n2.  The
// inverse runs the Gentleman-Sande butterflies in the opposite stage order,
// rows first, and folds n^{-1} into its final stage.
//
// A workgroup owns C columns (or rows) of S = 2^LOGS elements.  Each thread
// holds E = 2^LOGE elements in registers and runs up to LOGE stages between
// LDS exchanges; a round's LOGE-bit window of the local index selects which
// elements a thread holds.  Values stay lazily reduced: [0, 4q) in the
// forward direction, [0, 2q) in the inverse, canonical at the end.
// The butterfly core of one pass over the C columns (rows) c0 .. c0+C-1 of
// one limb: reads din (PRO: any uint64, reduced first), runs the pass's
// stages and hands every final value to emit(k, pos, y), k in [0, E) being
// the thread's ordinal of that element (the same position for every call
// from the same thread).
template <int LOGS, int LOGE, int C, bool COLPASS, bool INV, bool PRO, bool IN_LOOP = false, int NB = 1,
          bool LDS_IN = false, class Emit>
__device__ __forceinline__ void pass_core(const u64 *__restrict__ din, int c0, int logn, int mod, double q,
                                          double qinv, const double *__restrict__ twq,
                                          const double2 *__restrict__ twlast,
                                          double *lds, Emit &&emit, u32 gal = 0, double cq = 0.0,
                                          const double2 *twrow = nullptr, const u64 *din2 = nullptr,
                                          double2 c2 = double2{0.0, 0.0}) {
    constexpr int S = 1 << LOGS, E = 1 << LOGE, TPC = S / E, NT = C * TPC;
    constexpr int NR = (LOGS + LOGE - 1) / LOGE;
    static_assert(!PRO || (COLPASS && !INV), "the prologue feeds the first pass of the forward transform");
    static_assert(!LDS_IN || (!COLPASS && INV), "an LDS-resident tile feeds the first pass of the inverse");
    constexpr int SP = S + (S >> 4) + 1;
    constexpr bool FINAL = (INV == COLPASS);
    const double two_q = 2.0 * q;
    const int ncol = 1 << (logn - LOGS);
    // NB > 1: the workgroup holds NB groups of NT threads, each running this
    // pass on its own polynomial over the same rows, with its own LDS region
    int tid = NB > 1 ? (int)(threadIdx.x % NT) : (int)threadIdx.x;
    // Called in a loop (the fused key-switch kernel runs one pass per digit),
    // the compiler would compute every thread-dependent address once, before
    // the loop, and keep them all live across it: 2 waves per SIMD instead of
    // 3 (5 for 4 elements per thread).  An opaque copy of the thread index
    // makes it recompute them in each pass.
    if constexpr (IN_LOOP) asm volatile("" : "+v"(tid));
    const int cl = COLPASS ? (tid % C) : (tid / TPC);
    const int tau = COLPASS ? (tid / C) : (tid % TPC);
    const int c = c0 + cl;
    const int g0 = COLPASS ? 0 : (logn - LOGS);
    const int cpart = COLPASS ? 0 : c;
    // positions within one limb fit 32 bits (n <= 2^17): offsets from a uniform base
    auto gaddr = [&](int r) -> u32 { return COLPASS ? (u32)(r * ncol + c) : (u32)(c * S + r); };
    auto lidx = [&](int cc, int r) -> int { return cc * SP + r + (r >> 4); };
    // A row pass of one wave per LDS region exchanges data within the wave
    // only: a wave's LDS operations complete in issue order, so ordering the
    // compiler's memory accesses is enough (no s_barrier)
    constexpr bool STAGED = (IN_LOOP || NB > 1) && !COLPASS;  // row twiddles staged in LDS (twrow)
    constexpr bool WAVE_SYNC = STAGED && NT == 64;
    auto sync = [] {
        if constexpr (WAVE_SYNC) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
    };

    // Twiddles come from the w/q table alone (8 bytes each instead of 16);
    // w = rint(w/q * q) is recovered exactly: |(w/q) q - w| <= w 2^-53 < 1/8
    // for w < 2^50, and the FMA rounds the exact product once.  A row pass
    // recovers w at each use.  A column pass uses only the first S entries of
    // its limb's table, the same for every column: they are staged in LDS as
    // {w, w/q} pairs once per workgroup (after the C*SP data words), so its
    // butterflies read them there with no recovery.
    double2 *twl = nullptr;
    if constexpr (COLPASS) {
        twl = reinterpret_cast<double2 *>(lds + ((C * SP + 1) & ~1));
        for (int i = tid; i < S; i += NT) {
            const double wq = twq[i];
            twl[i] = make_double2(__fma_rn(wq, q, C52) - C52, wq);
        }
        __syncthreads();
    }
    auto twid = [&](int idx) -> double2 {
        if constexpr (COLPASS) {
            return twl[idx];
        } else {
            const double wq = twq[idx];
            return make_double2(__fma_rn(wq, q, C52) - C52, wq);
        }
    };
    // twiddle of stage s (global stage g) for local position r.  A row pass run
    // several times over the same rows (the fused key switch: one pass per
    // digit; NB > 1: one pass per polynomial of the workgroup) reads them from
    // twrow, the rows' {w, w/q} pairs staged in LDS once by the caller at
    // local index (1 << s) + (r >> (LOGS - s)).
    auto twid_at = [&](int s, int g, int r) -> double2 {
        if constexpr (STAGED) {
            return twrow[cl * S + (1 << s) + (r >> (LOGS - s))];
        } else {
            return twid((1 << g) + (cpart << s) + (r >> (LOGS - s)));
        }
    };
    double x[E];
    // A forward row pass of 256 points, 4 per thread, one row per wave, ends
    // its third round holding 16 h + 4 k + l in lane 4 h + l, register k, and
    // starts its fourth holding it in lane 4 h + k, register l: a transpose
    // inside each quad of lanes, done with DPP moves instead of LDS.
    constexpr bool QUADX = !COLPASS && !INV && LOGS == 8 && LOGE == 2 && TPC % 64 == 0;

#pragma unroll
    for (int rho = 0; rho < NR; rho++) {
        const int w = INV ? min(rho * LOGE, LOGS - LOGE) : max(LOGS - (rho + 1) * LOGE, 0);
        const int lo = tau & ((1 << w) - 1), hi = tau >> w;
        const int rbase = (hi << (w + LOGE)) | lo;
        const bool direct = COLPASS || w >= 3;
        // ---- load
        if (rho == 0) {
            if (PRO) {
                // the input limb's residues mod cq, taken in (-cq/2, cq/2) when cq > 0,
                // plus din2 * c2 when din2 is set: [0, q) + (0, 2q), below 4q, which
                // the forward butterflies take as it is
#pragma unroll
                for (int k = 0; k < E; k++) {
                    double v = u2d(din[gaddr(rbase | (k << w))]);
                    if (v > 0.5 * cq) v -= cq;
                    x[k] = red_any(v, q, qinv);
                    if (din2) x[k] += mm_lazy(u2d(din2[gaddr(rbase | (k << w))]), c2.x, c2.y, q);
                }
            } else if (direct) {
                if (gal > 1) {
#pragma unroll
                    for (int k = 0; k < E; k++) x[k] = u2d(din[gal_src(gaddr(rbase | (k << w)), logn, gal)]);
                } else {
#pragma unroll
                    for (int k = 0; k < E; k++) x[k] = u2d(din[gaddr(rbase | (k << w))]);
                }
            } else {
                // rows are contiguous: the tile is C*S consecutive words (LDS_IN:
                // the caller has put the tile in LDS already)
                if constexpr (!LDS_IN) {
                    const u64 *tile = din + (u32)(c0 * S);
                    if (gal > 1) {
                        for (int i = tid; i < C * S; i += NT)
                            lds[lidx(i / S, i % S)] = u2d(din[gal_src((u32)(c0 * S + i), logn, gal)]);
                    } else {
                        for (int i = tid; i < C * S; i += NT) lds[lidx(i / S, i % S)] = u2d(tile[i]);
                    }
                }
                sync();
#pragma unroll
                for (int k = 0; k < E; k++) x[k] = lds[lidx(cl, rbase | (k << w))];
            }
        } else if (!(QUADX && rho == NR - 1)) {
#pragma unroll
            for (int k = 0; k < E; k++) x[k] = lds[lidx(cl, rbase | (k << w))];
        }
        // ---- butterflies
        if (!INV) {
            const int s_begin = rho * LOGE, s_end = min((rho + 1) * LOGE, LOGS);
#pragma unroll
            for (int s = s_begin; s < s_end; s++) {
                const int kb = (LOGS - 1 - s) - w;
                const int g = g0 + s;
#pragma unroll
                for (int k = 0; k < E; k++) {
                    if (k & (1 << kb)) continue;
                    const int k2 = k | (1 << kb);
                    const int r = rbase | (k << w);
                    const double2 W = twid_at(s, g, r);
                    double u = x[k];
                    u = u >= two_q ? u - two_q : u;
                    const double v = mm_lazy(x[k2], W.x, W.y, q);
                    x[k] = u + v;
                    x[k2] = u - v + two_q;
                }
            }
        } else {
            const int b_begin = rho * LOGE, b_end = min((rho + 1) * LOGE, LOGS);
#pragma unroll
            for (int b = b_begin; b < b_end; b++) {
                const int s = LOGS - 1 - b;
                const int kb = b - w;
                const int g = g0 + s;
#pragma unroll
                for (int k = 0; k < E; k++) {
                    if (k & (1 << kb)) continue;
                    const int k2 = k | (1 << kb);
                    const double sm = x[k] + x[k2];
                    const double d = x[k] - x[k2] + two_q;
                    if (FINAL && g == 0) {
                        const double2 N0 = twlast[2 * mod], N1 = twlast[2 * mod + 1];
                        x[k] = mm_lazy(sm, N0.x, N0.y, q);
                        x[k2] = mm_lazy(d, N1.x, N1.y, q);
                    } else {
                        const int r = rbase | (k << w);
                        const double2 W = twid_at(s, g, r);
                        x[k] = sm >= two_q ? sm - two_q : sm;
                        x[k2] = mm_lazy(d, W.x, W.y, q);
                    }
                }
            }
        }
        // ---- store
        if (rho == NR - 1) {
            if (FINAL) {
#pragma unroll
                for (int k = 0; k < E; k++) {
                    double v = x[k];
                    if (!INV) v = v >= two_q ? v - two_q : v;
                    x[k] = v >= q ? v - q : v;
                }
            }
            if (direct) {
#pragma unroll
                for (int k = 0; k < E; k++) emit(k, gaddr(rbase | (k << w)), x[k]);
            } else {
                sync();
#pragma unroll
                for (int k = 0; k < E; k++) lds[lidx(cl, rbase | (k << w))] = x[k];
                sync();
#pragma unroll
                for (int k = 0; k < E; k++) {
                    const int i = tid + k * NT;
                    emit(k, (u32)(c0 * S + i), lds[lidx(i / S, i % S)]);
                }
            }
        } else if (QUADX && rho == NR - 2) {
            quad_transpose(x);
        } else {
            sync();
#pragma unroll
            for (int k = 0; k < E; k++) lds[lidx(cl, rbase | (k << w))] = x[k];
            sync();
        }
    }
}

// Forward transform (Cooley-Tukey, merged psi twiddles): stage g pairs indices
// j, j + n/2^{g+1} with twiddle w[2^g + (j >> (logn - g))].  The first logn1
// stages act on columns {c + n2 r}, the rest on contiguous rows of n2.  The
// inverse runs the Gentleman-Sande butterflies in the opposite stage order,
// rows first, and folds n^{-1} into its final stage.
//
// A workgroup owns C columns (or rows) of S = 2^LOGS elements.  Each thread
// holds E = 2^LOGE elements in registers and runs up to LOGE stages between
// LDS exchanges; a round's LOGE-bit window of the local index selects which
// elements a thread holds.  Values stay lazily reduced: [0, 4q) in the
// forward direction, [0, 2q) in the inverse, canonical at the end.
//
// NB > 1 (row passes, C rows per wave): the workgroup's NB waves take NB
// polynomials of the same limb over the same rows, and the rows' twiddles
// are staged in LDS once for all of them; a wave past the last polynomial
// repeats it and stores nothing.
template <int LOGS, int LOGE, int C, bool COLPASS, bool INV, bool FUSE, int NB = 1>
__global__ void __launch_bounds__(NB * C * (1 << (LOGS - LOGE)))
    ntt_pass(u64 *__restrict__ base, size_t poly_stride, int limbs, int polys, LimbMap map, int logn,
             const double2 *__restrict__ mq, const double *__restrict__ twqtab,
             const double2 *__restrict__ twlast, const NttFuse fz, const u64 *__restrict__ src, size_t src_stride,
             u32 gal) {
    constexpr int S = 1 << LOGS, NT = C * (S >> LOGE);
    constexpr int SP = S + (S >> 4) + 1;
    constexpr int REGION = ((C * SP + 1) & ~1);
    static_assert(NB == 1 || (!COLPASS && NT == 64), "shared-twiddle row passes: one wave per polynomial");
    __shared__ __align__(16) double lds[NB * REGION + (COLPASS ? 2 * S : 0)];
    __shared__ double2 twr[NB > 1 ? C * S : 1];

    const int job = blockIdx.y;
    const int slot = job / limbs, t = job - slot * limbs;
    const int wv = NB > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / NT)) : 0;
    const bool live = slot * NB + wv < polys;
    const int p = live ? slot * NB + wv : polys - 1;
    const int mod = map(t);
    const size_t n = (size_t)1 << logn;
    u64 *data = base + (size_t)p * poly_stride + (size_t)t * n;
    constexpr bool FIRST = (COLPASS != INV);  // the pass that runs first reads the input
    const u64 *din = (FIRST && src) ? src + (size_t)p * src_stride + (size_t)t * n : data;
    const double q = mq[mod].x, qinv = mq[mod].y;
    const double *twq = twqtab + (size_t)mod * n;
    if constexpr (NB > 1) {
        // row c0 + cl, stage s: table entry 2^(logn - LOGS + s) + ((c0 + cl) << s) + j,
        // staged at cl S + 2^s + j (entry 0 of each row unused)
        const int g0 = logn - LOGS;
        for (int i = threadIdx.x; i < C * S; i += NB * NT) {
            const int cl = i / S, li = i % S;
            if (li == 0) continue;
            const int st = 31 - __clz(li);
            const double wq = twq[(1 << (g0 + st)) + (((int)blockIdx.x * C + cl) << st) + (li - (1 << st))];
            twr[i] = make_double2(__fma_rn(wq, q, C52) - C52, wq);
        }
        __syncthreads();
    }
    double *ldsw = lds + wv * REGION;
    constexpr bool PRO = FUSE && COLPASS && !INV;   // prologue: broadcast-reduce one limb
    constexpr bool EPI = FUSE && !COLPASS && !INV;  // epilogue: (x - y) * c (+ add)
    const int c0 = blockIdx.x * C;
    const u32 g = (FIRST && src) ? gal : 0;  // automorphism applied while reading the input
    if constexpr (EPI) {
        const size_t pb = (size_t)(p >> 1), pk = (size_t)(p & 1);
        u64 *pout = fz.out + pb * fz.out_stride + pk * fz.out_off + (size_t)t * n;
        const u64 *px = fz.x + pb * fz.x_stride + pk * fz.x_off + (size_t)t * n;
        const u64 *padd = nullptr, *padd2 = nullptr;
        if (fz.add && (fz.add_mask >> pk & 1)) padd = fz.add + pb * fz.add_stride + pk * fz.add_off + (size_t)t * n;
        if (fz.add2 && (fz.add2_mask >> pk & 1))
            padd2 = fz.add2 + pb * fz.add2_stride + pk * fz.add2_off + (size_t)t * n;
        const double ec = fz.c.v[t], ecq = fz.c.vq[t];
        const double pc = fz.c2.v[t], pcq = fz.c2.vq[t];
        const bool pre = fz.pre, sub2 = fz.add2_sub;
        const u64 *pxm = fz.xmul ? fz.xmul + (size_t)t * n : nullptr;
        const u32 ag = fz.add_gal;
        pass_core<LOGS, LOGE, C, COLPASS, INV, false, false, NB>(din, c0, logn, mod, q, qinv, twq, twlast, ldsw,
                                                                 [&](int, u32 pos, double y) {
            if (!live) return;
            double r;
            if (pre) {
                // (x * c2 + add - y) * c
                double xv = red1(mm_lazy(u2d(px[pos]), pc, pcq, q), q);
                if (padd) xv = red1(xv + u2d(padd[ag > 1 ? gal_src(pos, logn, ag) : pos]), q);
                r = red1(mm_lazy(xv - y + q, ec, ecq, q), q);
            } else {
                double xv = u2d(px[pos]);
                if (pxm) xv = pos1(mm_signed(xv, u2d(pxm[pos]), q, qinv), q);  // slot-wise plaintext product
                r = red1(mm_lazy(xv - y + q, ec, ecq, q), q);
                if (padd) r = red1(r + u2d(padd[ag > 1 ? gal_src(pos, logn, ag) : pos]), q);
            }
            if (padd2) r = sub2 ? pos1(r - u2d(padd2[pos]), q) : red1(r + u2d(padd2[pos]), q);
            pout[pos] = d2u(r);
        }, 0, 0.0, twr);
    } else if constexpr (PRO) {
        const u64 *src2 = fz.src2 ? fz.src2 + (size_t)p * fz.src2_stride + (size_t)t * n : nullptr;
        pass_core<LOGS, LOGE, C, COLPASS, INV, true>(fz.src + (size_t)p * fz.src_stride, c0, logn, mod, q, qinv,
                                                     twq, twlast, ldsw,
                                                     [&](int, u32 pos, double y) { data[pos] = d2u(y); }, 0,
                                                     fz.pro_q, nullptr, src2,
                                                     make_double2(fz.c2.v[t], fz.c2.vq[t]));
    } else {
        pass_core<LOGS, LOGE, C, COLPASS, INV, false, false, NB>(
            din, c0, logn, mod, q, qinv, twq, twlast, ldsw,
            [&](int, u32 pos, double y) {
                if (live) data[pos] = d2u(y);
            },
            g, 0.0, twr);
    }
}

// Key-switch ModUp tail: the forward row pass of every digit's extended limb
// t fused with the inner product against the switching key,
//   accb[t] = sum_j X_j[t] kb_j[t],  acca[t] = sum_j X_j[t] ka_j[t],
// X_j[t] = d[t] for the digit that holds limb t, else the row-pass output of
// ext[j][t] (which has had its column pass).  One workgroup per (slot of NB
// batch entries, limb, tile of C rows); the extended limbs never go back to
// HBM in the evaluation domain.  Workgroups are dealt to the 8 XCDs
// round-robin, so the workgroup index is decoded as (xcd, then per-XCD
// sequence): the batch slots of one (limb, tile) run back to back on one XCD
// and read that tile's key words from its L2.  With NB > 1 (one row), the NB
// waves of a workgroup run NB batch entries over the same row: the row's
// twiddles and each digit's key words are staged in LDS once for all of them.
// With a.inv_p, the outputs of the special-prime limbs (t > level) also get
// the inverse transform's row pass, ModDown's first step, before they are
// stored: the same lazily reduced values that pass writes on its own.
template <int LOGS, int LOGE, int C, int NB>
__global__ void __launch_bounds__(NB * C * (1 << (LOGS - LOGE)), (LOGE == 2 ? 6 : 1))  // 4 elements: 78 VGPRs
    ntt_row_ip(const IPArgs a, int logn, const double2 *__restrict__ mq, const double *__restrict__ twqtab,
               const double *__restrict__ twqinv, const double2 *__restrict__ twlast) {
    constexpr int S = 1 << LOGS, E = 1 << LOGE, NT = C * (S / E), NALL = NB * NT;
    constexpr int SP = S + (S >> 4) + 1;
    static_assert(NB == 1 || (C == 1 && NT == 64 && LOGS - LOGE >= 3),
                  "batch-shared workgroups: one row per wave, first round read directly");
    __shared__ double lds[NB * C * SP];
    __shared__ double2 twr[C * S];  // the rows' forward twiddles {w, w/q}, shared by the digits' passes
    __shared__ double keyl[NB > 1 ? 2 * C * S : 2];  // NB > 1: the digit's key words kb, ka of the rows
    __shared__ double2 twi[NB > 1 ? C * S : 1];      // NB > 1 and a.inv_p: the rows' inverse twiddles
    const size_t n = (size_t)1 << logn;
    const int tiles = (int)(n >> LOGS) / C;
    const int slots = (a.B + NB - 1) / NB;
    const int wg = blockIdx.x, xcd = wg & 7, seq = wg >> 3;
    const int gl = seq / slots, slot = seq - gl * slots;
    const int g = gl * 8 + xcd;
    if (g >= a.E * tiles) return;
    // wave wv of the workgroup takes batch entry slot * NB + wv; a wave past
    // the batch end repeats the last entry (every wave must reach the
    // workgroup barriers) and stores nothing
    const int wv = NB > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x / NT)) : 0;
    const bool live = slot * NB + wv < a.B;
    const int bi = live ? slot * NB + wv : a.B - 1;
    const int t = g / tiles, c0 = (g - t * tiles) * C;
    const int mod = t <= a.level ? t : a.nq + (t - a.level - 1);
    const int kl = t <= a.level ? t : a.lmax_key + 1 + (t - a.level - 1);
    const double q = mq[mod].x, qinv = mq[mod].y;
    const double *twq = twqtab + (size_t)mod * n;
    const int own = (t <= a.level) ? t / a.alpha : -1;  // digit holding limb t, if any
    const int tall = threadIdx.x, tid = NB > 1 ? (int)(threadIdx.x % NT) : (int)threadIdx.x;
    const bool invp = a.inv_p && t > a.level;
    const double *twqi = twqinv + (size_t)mod * n;
    // row c0 + cl, stage s (global stage logn - LOGS + s) uses table entry
    // 2^(logn - LOGS + s) + ((c0 + cl) << s) + (r >> (LOGS - s)); staged at
    // cl S + 2^s + (r >> (LOGS - s)), entry 0 of each row unused
    auto stage = [&](double2 *dst, const double *tab) {
        const int g0 = logn - LOGS;
        for (int i = tall; i < C * S; i += NALL) {
            const int cl = i / S, li = i % S;
            if (li == 0) continue;
            const int st = 31 - __clz(li);
            const double wq = tab[(1 << (g0 + st)) + ((c0 + cl) << st) + (li - (1 << st))];
            dst[i] = make_double2(__fma_rn(wq, q, C52) - C52, wq);
        }
    };
    const bool fwd_staged = a.beta > (own >= 0 ? 1 : 0);
    if (fwd_staged) stage(twr, twq);
    if constexpr (NB > 1)
        if (invp) stage(twi, twqi);
    if (fwd_staged || (NB > 1 && invp)) __syncthreads();
    double sb[E], sa[E];
#pragma unroll
    for (int k = 0; k < E; k++) sb[k] = sa[k] = 0.0;
    for (int j = 0; j < a.beta; j++) {
        const u64 *kb = a.key + (((size_t)j * 2 + 0) * a.Ek + kl) * n;
        const u64 *ka = a.key + (((size_t)j * 2 + 1) * a.Ek + kl) * n;
        if constexpr (NB > 1) {
            __syncthreads();  // every wave is done with the previous digit's key words and row data
            for (int i = tall; i < C * S; i += NALL) {
                keyl[i] = u2d(kb[(u32)(c0 * S + i)]);
                keyl[C * S + i] = u2d(ka[(u32)(c0 * S + i)]);
            }
            __syncthreads();
        }
        // NB == 1: this digit's key words, read where the pass hands over its
        // outputs (held across the pass they would cost 4E registers).
        // Products in (-0.75q, 0.75q) accumulate unreduced: exact while the
        // sums stay below 2^53 in magnitude (the library allows at most 8
        // digits; a reduction every 8 keeps any count safe)
        auto acc = [&](int k, u32 pos, double x) {
            if constexpr (NB > 1) {
                const int r = (int)(pos - (u32)(c0 * S));
                sb[k] += mm_signed(x, keyl[r], q, qinv);
                sa[k] += mm_signed(x, keyl[C * S + r], q, qinv);
            } else {
                sb[k] += mm_signed(x, u2d(kb[pos]), q, qinv);
                sa[k] += mm_signed(x, u2d(ka[pos]), q, qinv);
            }
        };
        if (j == own) {
            const u64 *xs = a.d + bi * a.sd + (size_t)t * n;
            double xv[E];
            if (a.gal > 1) {
#pragma unroll
                for (int k = 0; k < E; k++) xv[k] = u2d(xs[gal_src((u32)(c0 * S + tid + k * NT), logn, a.gal)]);
            } else {
#pragma unroll
                for (int k = 0; k < E; k++) xv[k] = u2d(xs[(u32)(c0 * S + tid + k * NT)]);
            }
#pragma unroll
            for (int k = 0; k < E; k++) acc(k, (u32)(c0 * S + tid + k * NT), xv[k]);
        } else {
            if constexpr (NB == 1) __syncthreads();  // the previous digit's last LDS reads are done
            pass_core<LOGS, LOGE, C, false, false, false, true, NB>(
                a.ext + bi * a.sext + ((size_t)j * a.E + t) * n, c0, logn, mod, q, qinv, twq, twlast,
                lds + wv * (C * SP), acc, 0, 0.0, twr);
        }
        if ((j & 7) == 7) {
#pragma unroll
            for (int k = 0; k < E; k++) {
                sb[k] = red_any(sb[k], q, qinv);
                sa[k] = red_any(sa[k], q, qinv);
            }
        }
    }
    if (!live) return;  // NB > 1: only wave-level synchronisation follows
    u64 *ob = a.accb + bi * a.sacc + (size_t)t * n, *oa = a.acca + bi * a.sacc + (size_t)t * n;
    if (invp) {
        // each output row through the inverse row pass: the reduced sums go
        // into this wave's LDS tile, where that pass's first round reads them
        double *ldsw = lds + wv * (C * SP);
        auto region_sync = [] {
            if constexpr (NB > 1) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else {
                __syncthreads();
            }
        };
        auto inv_store = [&](const double(&sv)[E], u64 *o) {
            region_sync();  // earlier readers of the tile are done
#pragma unroll
            for (int k = 0; k < E; k++) {
                const int i = tid + k * NT;
                ldsw[(i / S) * SP + i % S + ((i % S) >> 4)] = red_any(sv[k], q, qinv);
            }
            pass_core<LOGS, LOGE, C, false, true, false, false, NB, true>(
                nullptr, c0, logn, mod, q, qinv, twqi, twlast, ldsw, [&](int, u32 pos, double y) { o[pos] = d2u(y); },
                0, 0.0, twi);
        };
        inv_store(sb, ob);
        inv_store(sa, oa);
        return;
    }
#pragma unroll
    for (int k = 0; k < E; k++) {
        const u32 pos = (u32)(c0 * S + tid + k * NT);
        ob[pos] = d2u(red_any(sb[k], q, qinv));
        oa[pos] = d2u(red_any(sa[k], q, qinv));
    }
}

template <int LOGS, int LOGE, int C, int NB = 1>
static void launch_row_ip(const DevTables &T, const IPArgs &a, hipStream_t s) {
    static_assert(NB * C * (1 << (LOGS - LOGE)) <= 1024, "workgroup larger than 1024 threads");
    const int tiles = (1 << (T.logn - LOGS)) / C;
    const int groups = a.E * tiles;
    const unsigned blocks = (unsigned)(((groups + 7) / 8) * 8) * (unsigned)((a.B + NB - 1) / NB);
    hipLaunchKernelGGL((ntt_row_ip<LOGS, LOGE, C, NB>), dim3(blocks), dim3(NB * C * (1 << (LOGS - LOGE))), 0, s, a,
                       T.logn, T.mq, T.twq_fwd, T.twq_inv, T.tw_last);
}


template <int LOGS, int LOGE, int C, bool COLPASS, bool INV, int NB = 1>
static void launch_pass(const DevTables &T, const LimbBatch &b, hipStream_t s, const NttFuse *f = nullptr) {
    static_assert(NB * C * (1 << (LOGS - LOGE)) <= 1024, "workgroup larger than 1024 threads");
    const int logn = T.logn;
    const int blocks = (1 << (logn - LOGS)) / C;
    dim3 grid(blocks, b.limbs * ((b.polys + NB - 1) / NB));
    dim3 block(NB * C * (1 << (LOGS - LOGE)));
    const double *twq = INV ? T.twq_inv : T.twq_fwd;
    if (f && !INV && (COLPASS ? f->pro : f->epi))
        hipLaunchKernelGGL((ntt_pass<LOGS, LOGE, C, COLPASS, INV, true, NB>), grid, block, 0, s, b.base,
                           b.poly_stride, b.limbs, b.polys, b.map, logn, T.mq, twq, T.tw_last, *f, b.src,
                           b.src_stride, b.gal);
    else
        hipLaunchKernelGGL((ntt_pass<LOGS, LOGE, C, COLPASS, INV, false, NB>), grid, block, 0, s, b.base,
                           b.poly_stride, b.limbs, b.polys, b.map, logn, T.mq, twq, T.tw_last, NttFuse{}, b.src,
                           b.src_stride, b.gal);
}

// entries per workgroup of the shared tiles (row passes: polynomials, fused
// key switch: batch entries): 4 or 2, the larger that leaves at most B/8
// idle waves (a ragged last slot), else 1
static int share_of(int B) {
    for (int nb = 4; nb > 1; nb >>= 1)
        if (B >= nb && ((B + nb - 1) / nb * nb - B) * 8 <= B) return nb;
    return 1;
}

// tile variants: (elements per thread 2^LOGE, columns per workgroup C)
//   passes of 2^8 and 2^9 points: 0 (16, 16), 1 (8, 32) / (16, 32), 2 (8, 16), 3 (8, 8),
//   4: row passes of 2^8 points, (4, 1) forward and (8, 2) inverse per wave,
//   with up to 4 polynomials per workgroup sharing the rows' staged
//   twiddles; column passes as 3
//   smaller passes: one fixed tile
template <int LOGS, bool COLPASS, bool INV>
static void pass_variant(const DevTables &T, const LimbBatch &b, hipStream_t s, const NttFuse *f, int v) {
    if constexpr (LOGS == 8 || LOGS == 9) {
        switch (v) {
        case 1: launch_pass<LOGS, (LOGS == 8 ? 3 : 4), 32, COLPASS, INV>(T, b, s, f); return;
        case 2: launch_pass<LOGS, 3, 16, COLPASS, INV>(T, b, s, f); return;
        case 3: launch_pass<LOGS, 3, 8, COLPASS, INV>(T, b, s, f); return;
        case 4:
            if constexpr (LOGS == 8 && !COLPASS) {
                // forward: one row of 4 per lane (its last exchange in DPP);
                // inverse: two rows of 8 per lane
                constexpr int E2 = INV ? 3 : 2, CR = INV ? 2 : 1;
                switch (share_of(b.polys)) {
                case 4: launch_pass<8, E2, CR, false, INV, 4>(T, b, s, f); return;
                case 2: launch_pass<8, E2, CR, false, INV, 2>(T, b, s, f); return;
                default: launch_pass<8, E2, CR, false, INV>(T, b, s, f); return;
                }
            } else {
                launch_pass<LOGS, 3, 8, COLPASS, INV>(T, b, s, f);
                return;
            }
        default: launch_pass<LOGS, 4, 16, COLPASS, INV>(T, b, s, f); return;
        }
    } else if constexpr (LOGS == 7) {
        launch_pass<7, 4, 16, COLPASS, INV>(T, b, s, f);
    } else if constexpr (LOGS == 6) {
        launch_pass<6, 3, 16, COLPASS, INV>(T, b, s, f);
    } else {
        launch_pass<5, 4, (COLPASS ? 16 : 32), COLPASS, INV>(T, b, s, f);
    }
}

// pass 0 runs first: the column pass (log n1 = ceil(logn/2) points) forward,
// the row pass (floor(logn/2) points) inverse
template <int L1, int L2>
static void pass_dispatch(const DevTables &T, const LimbBatch &b, bool inv, int pass, hipStream_t s, const NttFuse *f,
                          int v) {
    if (!inv) {
        if (pass == 0) pass_variant<L1, true, false>(T, b, s, f, v);
        else pass_variant<L2, false, false>(T, b, s, f, v);
    } else {
        if (pass == 0) pass_variant<L2, false, true>(T, b, s, f, v);
        else pass_variant<L1, true, true>(T, b, s, f, v);
    }
}

static void run_pass(const DevTables &T, const LimbBatch &b, bool inv, int pass, hipStream_t s, const NttFuse *f,
                     int v) {
    if (b.limbs * b.polys == 0) return;
    switch (T.logn) {
    case 10: pass_dispatch<5, 5>(T, b, inv, pass, s, f, v); break;
    case 11: pass_dispatch<6, 5>(T, b, inv, pass, s, f, v); break;
    case 12: pass_dispatch<6, 6>(T, b, inv, pass, s, f, v); break;
    case 13: pass_dispatch<7, 6>(T, b, inv, pass, s, f, v); break;
    case 14: pass_dispatch<7, 7>(T, b, inv, pass, s, f, v); break;
    case 15: pass_dispatch<8, 7>(T, b, inv, pass, s, f, v); break;
    case 16: pass_dispatch<8, 8>(T, b, inv, pass, s, f, v); break;
    case 17: pass_dispatch<9, 8>(T, b, inv, pass, s, f, v); break;
    default: break;
    }
}

// tiles of the fused row pass + inner product, (elements per thread, rows per
// workgroup) for passes of 2^8 points: 0 (8, 16), 1 (8, 8), 2 (8, 4), 3 (8, 2),
// 4 (4, 4), 5 (4, 2), 6 (4, 1), 7 (4, 1) with up to 4 batch entries per
// workgroup sharing the staged twiddles and key words; smaller passes: one
// fixed tile
template <int LOGS>
static void row_ip_variant(const DevTables &T, const IPArgs &a, hipStream_t s, int v) {
    if constexpr (LOGS == 8) {
        switch (v) {
        case 1: launch_row_ip<8, 3, 8>(T, a, s); return;
        case 2: launch_row_ip<8, 3, 4>(T, a, s); return;
        case 3: launch_row_ip<8, 3, 2>(T, a, s); return;
        case 4: launch_row_ip<8, 2, 4>(T, a, s); return;
        case 5: launch_row_ip<8, 2, 2>(T, a, s); return;
        case 6: launch_row_ip<8, 2, 1>(T, a, s); return;
        case 7:
            switch (share_of(a.B)) {
            case 4: launch_row_ip<8, 2, 1, 4>(T, a, s); return;
            case 2: launch_row_ip<8, 2, 1, 2>(T, a, s); return;
            default: launch_row_ip<8, 2, 1>(T, a, s); return;
            }
        default: launch_row_ip<8, 3, 16>(T, a, s); return;
        }
    } else if constexpr (LOGS == 7) {
        launch_row_ip<7, 3, 4>(T, a, s);
    } else if constexpr (LOGS == 6) {
        launch_row_ip<6, 3, 8>(T, a, s);
    } else {
        launch_row_ip<5, 3, 16>(T, a, s);
    }
}

void k_ntt_row_ip(const DevTables &T, const IPArgs &a, hipStream_t s) {
    if (a.E == 0 || a.B == 0) return;
    const int v = T.row_ip_variant;
    switch (T.logn) {
    case 10: case 11: row_ip_variant<5>(T, a, s, v); break;
    case 12: case 13: row_ip_variant<6>(T, a, s, v); break;
    case 14: case 15: row_ip_variant<7>(T, a, s, v); break;
    case 16: case 17: row_ip_variant<8>(T, a, s, v); break;
    default: break;
    }
}

void k_ntt_pass(const DevTables &T, const LimbBatch &b, bool inverse, int pass, hipStream_t s) {
    run_pass(T, b, inverse, pass, s, nullptr, T.ntt_variant[inverse][pass]);
}

void k_ntt_pass_variant(const DevTables &T, const LimbBatch &b, bool inverse, int pass, int variant, hipStream_t s) {
    run_pass(T, b, inverse, pass, s, nullptr, variant);
}

void k_ntt_fused(const DevTables &T, const LimbBatch &b, const NttFuse &f, int pass, hipStream_t s) {
    run_pass(T, b, false, pass, s, &f, T.ntt_variant[0][pass]);
}

void k_ntt(const DevTables &T, const LimbBatch &b, bool inverse, hipStream_t s) {
    k_ntt_pass(T, b, inverse, 0, s);
    k_ntt_pass(T, b, inverse, 1, s);
}

// ------------------------------------------------------------------------
// elementwise kernels: grid.x covers n/2 pairs of coefficients, grid.y the limbs
// ------------------------------------------------------------------------
#define EW_PROLOGUE                                                       \
    const int job = blockIdx.y;                                           \
    const int p = job / limbs, t = job - p * limbs;                       \
    const size_t n = (size_t)1 << logn;                                   \
    const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; \
    if (i >= n) return;

__global__ void ew_add(u64 *out, const u64 *a, const u64 *b, int limbs, size_t so, size_t sa, size_t sb, LimbMap map,
                       int logn, const u64 *qi, int sub) {
    EW_PROLOGUE
    const u64 q = qi[map(t)];
    const ulonglong2 va = *(const ulonglong2 *)(a + p * sa + t * n + i);
    const ulonglong2 vb = *(const ulonglong2 *)(b + p * sb + t * n + i);
    ulonglong2 r;
    if (sub) {
        r.x = va.x >= vb.x ? va.x - vb.x : va.x + (q - vb.x);
        r.y = va.y >= vb.y ? va.y - vb.y : va.y + (q - vb.y);
    } else {
        r.x = va.x + vb.x; r.x = r.x >= q ? r.x - q : r.x;
        r.y = va.y + vb.y; r.y = r.y >= q ? r.y - q : r.y;
    }
    *(ulonglong2 *)(out + p * so + t * n + i) = r;
}

__global__ void ew_add_scalar(u64 *data, int limbs, size_t stride, LimbMap map, int logn, const u64 *qi,
                              LimbScalars c) {
    EW_PROLOGUE
    const u64 q = qi[map(t)];
    const u64 k = (u64)c.v[t];
    u64 *ptr = data + p * stride + t * n + i;
    ulonglong2 v = *(ulonglong2 *)ptr;
    v.x += k; v.x = v.x >= q ? v.x - q : v.x;
    v.y += k; v.y = v.y >= q ? v.y - q : v.y;
    *(ulonglong2 *)ptr = v;
}

__global__ void ew_mul_scalar(u64 *out, const u64 *a, int limbs, size_t so, size_t sa, LimbMap map, int logn,
                              const double2 *mq, LimbScalars c) {
    EW_PROLOGUE
    const double q = mq[map(t)].x;
    const double w = c.v[t], wq = c.vq[t];
    const ulonglong2 v = *(const ulonglong2 *)(a + p * sa + t * n + i);
    ulonglong2 r;
    r.x = d2u(red1(mm_lazy(u2d(v.x), w, wq, q), q));
    r.y = d2u(red1(mm_lazy(u2d(v.y), w, wq, q), q));
    *(ulonglong2 *)(out + p * so + t * n + i) = r;
}

__global__ void ew_mul_pt(u64 *out, const u64 *a, const u64 *pt, int limbs, size_t so, size_t sa, LimbMap map,
                          int logn, const double2 *mq, const u64 *qi, int add) {
    EW_PROLOGUE
    const ulonglong2 v = *(const ulonglong2 *)(a + p * sa + t * n + i);
    const ulonglong2 m = *(const ulonglong2 *)(pt + t * n + i);
    ulonglong2 r;
    if (add) {
        const u64 q = qi[map(t)];
        r.x = v.x + m.x; r.x = r.x >= q ? r.x - q : r.x;
        r.y = v.y + m.y; r.y = r.y >= q ? r.y - q : r.y;
    } else {
        const double2 Q = mq[map(t)];
        r.x = d2u(pos1(mm_signed(u2d(v.x), u2d(m.x), Q.x, Q.y), Q.x));
        r.y = d2u(pos1(mm_signed(u2d(v.y), u2d(m.y), Q.x, Q.y), Q.x));
    }
    *(ulonglong2 *)(out + p * so + t * n + i) = r;
}

__global__ void ew_tensor(u64 *d, const u64 *a, const u64 *bb, int limbs, size_t sd, size_t sa, size_t sb, int logn,
                          const double2 *mq) {
    EW_PROLOGUE
    const double2 Q = mq[t];
    const size_t L = (size_t)limbs * n, o = t * n + i;
    const u64 *A = a + p * sa, *Bq = bb + p * sb;
    u64 *D = d + p * sd;
    const ulonglong2 A0 = *(const ulonglong2 *)(A + o), A1 = *(const ulonglong2 *)(A + L + o);
    const ulonglong2 B0 = *(const ulonglong2 *)(Bq + o), B1 = *(const ulonglong2 *)(Bq + L + o);
    ulonglong2 r0, r1, r2;
    {
        const double x0 = u2d(A0.x), x1 = u2d(A1.x), y0 = u2d(B0.x), y1 = u2d(B1.x);
        r0.x = d2u(pos1(mm_signed(x0, y0, Q.x, Q.y), Q.x));
        const double m = mm_signed(x0, y1, Q.x, Q.y) + mm_signed(x1, y0, Q.x, Q.y);  // (-1.5q, 1.5q)
        r1.x = d2u(red_any(m, Q.x, Q.y));
        r2.x = d2u(pos1(mm_signed(x1, y1, Q.x, Q.y), Q.x));
    }
    {
        const double x0 = u2d(A0.y), x1 = u2d(A1.y), y0 = u2d(B0.y), y1 = u2d(B1.y);
        r0.y = d2u(pos1(mm_signed(x0, y0, Q.x, Q.y), Q.x));
        const double m = mm_signed(x0, y1, Q.x, Q.y) + mm_signed(x1, y0, Q.x, Q.y);
        r1.y = d2u(red_any(m, Q.x, Q.y));
        r2.y = d2u(pos1(mm_signed(x1, y1, Q.x, Q.y), Q.x));
    }
    *(ulonglong2 *)(D + o) = r0;
    *(ulonglong2 *)(D + L + o) = r1;
    *(ulonglong2 *)(D + 2 * L + o) = r2;
}

// evaluation position i holds a(psi^{2 brev(i) + 1}); sigma_g reads position
// brev(((2 brev(i) + 1) g mod 2n - 1) / 2)
__global__ void ew_automorph(u64 *out, const u64 *in, int limbs, size_t so, size_t si, int logn, u32 g) {
    const int job = blockIdx.y;
    const int p = job / limbs, t = job - p * limbs;
    const size_t n = (size_t)1 << logn;
    const u32 i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[p * so + t * n + i] = in[p * si + t * n + gal_src(i, logn, g)];
}

// fast base conversion; grid.x over coefficients, grid.y over the batch,
// grid.z over groups of `tpg` targets.  y_i = [x_i * hinv_i]_{q_i} once per
// source, then for each target t: sum_i y_i * hmod[i][t] mod t.  Lazy products
// are < 2t and the sum is reduced only when more terms could leave the exact
// range of doubles: once at the end for small targets, every 3 terms near 2^50.
// The conversion constants are the same for every thread of a workgroup: they
// are read through restrict pointers, which the compiler serves from the
// scalar cache (no LDS staging, no barrier).
template <int NS>
__global__ void __launch_bounds__(256)
    ew_bconv(u64 *out, const u64 *__restrict__ src, BConvTab tab, const double2 *__restrict__ hmod,
             const double2 *__restrict__ hinv, int logn, size_t so, size_t si, const double2 *__restrict__ mq,
             int tpg) {
    // two adjacent coefficients per thread: 16-byte loads and stores, and
    // every (source, target) constant serves two products
    const size_t n = (size_t)1 << logn;
    const int j0 = blockIdx.z * tpg, j1 = min(j0 + tpg, tab.nt);
    const size_t c = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
    if (c >= n) return;
    const u64 *sb = src + blockIdx.y * si;
    u64 *ob = out + blockIdx.y * so;
    double y0[NS], y1[NS];
    // exact conversion (rounding ModDown): overflow counts u = floor(sum_i y_i / p_i)
    const bool exact = tab.rinv != nullptr;
    double v0 = 0.0, v1 = 0.0;
#pragma unroll
    for (int i = 0; i < NS; i++) {
        const double q = mq[tab.src_mod[i]].x;
        const double2 h = hinv[i];
        const ulonglong2 v = *(const ulonglong2 *)(sb + (size_t)i * n + c);
        const double a = tab.pre ? tab.pre[i] : 0.0;  // added before the product: x + a < 2q
        y0[i] = red1(mm_lazy(u2d(v.x) + a, h.x, h.y, q), q);
        y1[i] = red1(mm_lazy(u2d(v.y) + a, h.x, h.y, q), q);
        if (exact) {
            const double r = tab.rinv[i];
            v0 = __dadd_rn(v0, __dmul_rn(y0[i], r));
            v1 = __dadd_rn(v1, __dmul_rn(y1[i], r));
        }
    }
    const double u0 = floor(v0), u1 = floor(v1);  // 0 unless exact
    for (int j = j0; j < j1; j++) {
        const double2 Q = mq[tab.tgt_mod[j]];
        const double tq = Q.x;
        double b0 = tab.post ? tab.post[j] : 0.0, b1 = b0;
        if (exact) {
            // subtract u P: b + [u P]_t in [0, 2t), reduced once
            const double2 pm = tab.pmod[j];
            b0 = red1(b0 + red1(mm_lazy(u0, pm.x, pm.y, tq), tq), tq);
            b1 = red1(b1 + red1(mm_lazy(u1, pm.x, pm.y, tq), tq), tq);
        }
        // the sum starts at -b in (-tq, 0] and gains terms in (0, 2 tq).  From a
        // start in (-tq, tq), m terms keep it below (2m + 1) tq, exact while
        // that is at most 2^53: all NS terms for small targets, else 3 at a
        // time (every modulus is below 2^50 < 2^53 / 7), reduced in between
        double a0 = -b0, a1 = -b1;
        if (tq * (2 * NS + 1) <= C53) {
#pragma unroll
            for (int i = 0; i < NS; i++) {
                const double2 h = hmod[i * tab.nt + j];
                a0 += mm_lazy(y0[i], h.x, h.y, tq);
                a1 += mm_lazy(y1[i], h.x, h.y, tq);
            }
        } else {
#pragma unroll
            for (int i = 0; i < NS; i++) {
                const double2 h = hmod[i * tab.nt + j];
                a0 += mm_lazy(y0[i], h.x, h.y, tq);
                a1 += mm_lazy(y1[i], h.x, h.y, tq);
                if (i % 3 == 2 && i + 1 < NS) {
                    a0 = red_any(a0, tq, Q.y);
                    a1 = red_any(a1, tq, Q.y);
                }
            }
        }
        a0 = red_any(a0, tq, Q.y);
        a1 = red_any(a1, tq, Q.y);
        *(ulonglong2 *)(ob + (size_t)tab.tgt_slot[j] * n + c) = make_ulonglong2(d2u(a0), d2u(a1));
    }
}

__global__ void ew_check_range(const u64 *data, int limbs, size_t stride, int logn, const u64 *qi, int *flag) {
    EW_PROLOGUE
    const u64 q = qi[t];
    const ulonglong2 v = *(const ulonglong2 *)(data + p * stride + t * n + i);
    if (v.x >= q || v.y >= q) atomicOr(flag, 1);
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
static dim3 ew_grid(int logn, int jobs) { return dim3((unsigned)(((1u << logn) / 2 + 255) / 256), (unsigned)jobs); }

void k_add(const DevTables &T, u64 *out, const u64 *a, const u64 *b, int limbs, int polys, size_t so, size_t sa,
           size_t sb, LimbMap map, bool sub, hipStream_t s) {
    if (limbs * polys == 0) return;
    hipLaunchKernelGGL(ew_add, ew_grid(T.logn, limbs * polys), dim3(256), 0, s, out, a, b, limbs, so, sa, sb, map,
                       T.logn, T.qi, (int)sub);
}
void k_add_scalar(const DevTables &T, u64 *data, int limbs, int polys, size_t stride, LimbMap map,
                  const LimbScalars &c, hipStream_t s) {
    hipLaunchKernelGGL(ew_add_scalar, ew_grid(T.logn, limbs * polys), dim3(256), 0, s, data, limbs, stride, map,
                       T.logn, T.qi, c);
}
void k_mul_scalar(const DevTables &T, u64 *out, const u64 *a, int limbs, int polys, size_t so, size_t sa,
                  LimbMap map, const LimbScalars &c, hipStream_t s) {
    hipLaunchKernelGGL(ew_mul_scalar, ew_grid(T.logn, limbs * polys), dim3(256), 0, s, out, a, limbs, so, sa, map,
                       T.logn, T.mq, c);
}
// one thread per coefficient position of one limb of one polynomial: the nt
// term values are loaded once and every output's combination is accumulated
// lazily in [0, 2q); the constants are uniform across the workgroup.
template <int NT>
__global__ void __launch_bounds__(256) ew_lincomb(const LinComb a, const double2 *__restrict__ kt, int logn,
                                                  const double2 *__restrict__ mq) {
    const size_t n = (size_t)1 << logn;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int t = blockIdx.y, pb = blockIdx.z;  // limb; batch entry * 2 + polynomial
    const double q = mq[t].x, two_q = 2.0 * q;
    const size_t entry = (size_t)2 * a.limbs * n;
    const size_t off = (size_t)(pb >> 1) * entry + (size_t)(pb & 1) * a.limbs * n + (size_t)t * n + i;
    double x[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) x[j] = j < a.nt ? u2d(a.term[j][off]) : 0.0;
    for (int o = 0; o < a.nout; o++) {
        const double2 *kk = kt + (size_t)o * a.nt * a.limbs + t;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < NT; j++) {
            if (j < a.nt) {
                const double2 w = kk[(size_t)j * a.limbs];
                acc += mm_lazy(x[j], w.x, w.y, q);
                acc = acc >= two_q ? acc - two_q : acc;
            }
        }
        a.out[(size_t)o * a.B * entry + off] = d2u(red1(acc, q));
    }
}

void k_lincomb(const DevTables &T, const LinComb &a, hipStream_t s) {
    const dim3 grid((unsigned)(((1u << T.logn) + 255) / 256), (unsigned)a.limbs, (unsigned)(2 * a.B));
    if (a.nt <= 8) hipLaunchKernelGGL(ew_lincomb<8>, grid, dim3(256), 0, s, a, a.k, T.logn, T.mq);
    else if (a.nt <= 16) hipLaunchKernelGGL(ew_lincomb<16>, grid, dim3(256), 0, s, a, a.k, T.logn, T.mq);
    else if (a.nt <= 32) hipLaunchKernelGGL(ew_lincomb<32>, grid, dim3(256), 0, s, a, a.k, T.logn, T.mq);
    else hipLaunchKernelGGL(ew_lincomb<64>, grid, dim3(256), 0, s, a, a.k, T.logn, T.mq);
}

void k_mul_pt(const DevTables &T, u64 *out, const u64 *a, const u64 *pt, int limbs, int polys, size_t so, size_t sa,
              LimbMap map, bool add, hipStream_t s) {
    hipLaunchKernelGGL(ew_mul_pt, ew_grid(T.logn, limbs * polys), dim3(256), 0, s, out, a, pt, limbs, so, sa, map,
                       T.logn, T.mq, T.qi, (int)add);
}
void k_tensor(const DevTables &T, u64 *d, const u64 *a, const u64 *bb, int limbs, int batch, size_t sd, size_t sa,
              size_t sb, hipStream_t s) {
    hipLaunchKernelGGL(ew_tensor, ew_grid(T.logn, limbs * batch), dim3(256), 0, s, d, a, bb, limbs, sd, sa, sb, T.logn,
                       T.mq);
}
void k_automorph(const DevTables &T, u64 *out, const u64 *in, int limbs, int polys, size_t so, size_t si, u32 g,
                 hipStream_t s) {
    dim3 grid((unsigned)((1u << T.logn) / 256 > 0 ? (1u << T.logn) / 256 : 1), (unsigned)(limbs * polys));
    hipLaunchKernelGGL(ew_automorph, grid, dim3(256), 0, s, out, in, limbs, so, si, T.logn, g);
}
void k_bconv(const DevTables &T, u64 *out, const u64 *src, const BConvTab &tab, int batch, size_t so, size_t si,
             hipStream_t s) {
    // two coefficients per thread; split the targets into groups so small
    // batches still fill the chip
    const unsigned bx = ((1u << T.logn) / 2 + 255) / 256;
    const int blocks = (int)bx * batch;
    int groups = std::max(1, std::min(tab.nt, 2048 / std::max(blocks, 1)));
    const int tpg = (tab.nt + groups - 1) / groups;
    groups = (tab.nt + tpg - 1) / tpg;
    dim3 grid(bx, (unsigned)batch, (unsigned)groups);
#define BCONV_CASE(K)                                                                                       \
    case K:                                                                                                 \
        hipLaunchKernelGGL(ew_bconv<K>, grid, dim3(256), 0, s, out, src, tab, tab.hmod, tab.hinv, T.logn, so, si, \
                           T.mq, tpg);                                                                        \
        break;
    switch (tab.ns) {
        BCONV_CASE(1) BCONV_CASE(2) BCONV_CASE(3) BCONV_CASE(4) BCONV_CASE(5) BCONV_CASE(6) BCONV_CASE(7)
        BCONV_CASE(8) BCONV_CASE(9) BCONV_CASE(10) BCONV_CASE(11) BCONV_CASE(12) BCONV_CASE(13) BCONV_CASE(14)
        BCONV_CASE(15) BCONV_CASE(16)
    default: break;
    }
#undef BCONV_CASE
}
void k_check_range(const DevTables &T, const u64 *data, int limbs, int polys, size_t stride, int *flag,
                   hipStream_t s) {
    hipLaunchKernelGGL(ew_check_range, ew_grid(T.logn, limbs * polys), dim3(256), 0, s, data, limbs, stride, T.logn,
                       T.qi, flag);
}

}  // namespace ckr
