"""Slot-level shadow of the paper's circuits -- test infrastructure only.

Plain float64 vectors stand in for ciphertext slots: no encryption, no
noise, no levels.  Every function follows the paper's matrix operations and
algorithms step by step:
  * section 2.3 (row-by-row matrix encoding, MaskR/MaskC),
  * Algorithm TransR / TransC (section 2.3),
  * Appendix A (SumR, SumC, ReplR, ReplC),
  * Algorithm Rank (section 3.1), Order Statistic (section 3.2),
    Sorting (section 3.3), Tie-Correction Offset (section 4).
Rotations are cyclic over `slots` positions: x << k means new[j] = x[j+k].

The comparator is either the ideal function of Eq. (1) applied to the pair
(x, y), the f/g composite of section 2.2 applied to x - y, or the Chebyshev
interpolant of Eq. (1) on [-1, 1] (section 2.2).  A comparator spec is a
tuple (d_g, d_f) for the composite or (0, 0, D) for the Chebyshev
interpolant of degree 2^(D-1) - 1, whose evaluation takes D levels.
"""
import numpy as np
from numpy.polynomial import chebyshev as _cheb

F_COEF = (35 / 16, -35 / 16, 21 / 16, -5 / 16)
G_COEF = (4589 / 1024, -16577 / 1024, 25614 / 1024, -12860 / 1024)
# minimax composite (section 2.2's pointer to composite minimax approximations
# of the sign function): stage s is the odd degree-7 minimax approximation of
# 1 on the interval stage s-1 maps [2^-8.5, 1] onto, stage 0 on [2^-8.5, 1]
# itself; coefficients of x, x^3, x^5, x^7
MM_COEF = (
    (11.626630381861787, -68.36534054680979, 126.44790262989271, -69.67707957286088),
    (5.38484717173034, -7.907363201737443, 3.7393070660732937, -0.5295271268765817),
    (3.8547436306459173, -5.358791130620638, 2.7473565274453287, -0.4363096838044091),
    (2.363269725894833, -2.5537068630909263, 1.5095093062451124, -0.32798232661912397),
    (2.1876161909909757, -2.187742945230383, 1.3126373118789916, -0.3125105627390891),
)
MM_DESIGN_LO = 2.0 ** -8.5


def rot_left(x, k):
    return np.roll(x, -int(k))


def rot_right(x, k):
    return np.roll(x, int(k))


def log2i(N):
    return int(N).bit_length() - 1


def mask_row(x, N, r):
    m = np.zeros_like(x)
    m[r * N:(r + 1) * N] = 1.0
    return x * m


def mask_col(x, N, c):
    m = np.zeros_like(x)
    m[c:N * N:N] = 1.0
    return x * m


def trans_r(x, N, trace=None):
    for i in range(1, log2i(N) + 1):
        x = x + rot_right(x, N * (N - 1) >> i)
        if trace is not None:
            trace.append(x.copy())
    return mask_col(x, N, 0)


def trans_c(x, N, trace=None):
    for i in range(1, log2i(N) + 1):
        x = x + rot_left(x, N * (N - 1) >> i)
        if trace is not None:
            trace.append(x.copy())
    return mask_row(x, N, 0)


def sum_r(x, N):
    for i in range(log2i(N)):
        x = x + rot_left(x, N << i)
    return mask_row(x, N, 0)


def sum_c(x, N):
    for i in range(log2i(N)):
        x = x + rot_left(x, 1 << i)
    return mask_col(x, N, 0)


def repl_r(x, N):
    for i in range(log2i(N)):
        x = x + rot_right(x, N << i)
    return x


def repl_c(x, N):
    for i in range(log2i(N)):
        x = x + rot_right(x, 1 << i)
    return x


def cmp_ideal(x, y):
    """Eq. (1): 1 if x > y, 0.5 if x == y, 0 if x < y."""
    return np.where(x > y, 1.0, np.where(x == y, 0.5, 0.0))


def poly7(x, a):
    return a[0] * x + a[1] * x ** 3 + a[2] * x ** 5 + a[3] * x ** 7


def cmp_composite(d, dg, df):
    """(f^{d_f}(g^{d_g}(d)) + 1) / 2 on the difference d = x - y (section 2.2)."""
    for _ in range(dg):
        d = poly7(d, G_COEF)
    for _ in range(df):
        d = poly7(d, F_COEF)
    return (d + 1.0) / 2.0


def cheb_step_coeffs(D):
    """Chebyshev coefficients of the interpolant of Eq. (1) (as a function
    of d = x - y) at the 2M = 2^(D-1) Chebyshev nodes of [-1, 1]: degree
    2M - 1, c_0 = 1/2, c_k = 0 for even k > 0 and, for odd k,
    c_k = (-1)^((k-1)/2) / (2M sin(pi k / 4M)) (the node sum in closed form)."""
    M = 1 << (D - 2)
    c = np.zeros(2 * M)
    c[0] = 0.5
    k = np.arange(1, 2 * M, 2)
    c[1::2] = np.where((k - 1) // 2 % 2 == 0, 1.0, -1.0) / (2 * M * np.sin(np.pi * k / (4 * M)))
    return c


def is_cheb(cmp):
    return len(cmp) >= 3 and cmp[2] > 0


def is_minimax(cmp):
    return len(cmp) == 4 and cmp[3] > 0


def sign_minimax(d, k):
    """the first k stages of the minimax composite on d"""
    for a in MM_COEF[:k]:
        d = poly7(d, a)
    return d


def cmp_of(d, cmp):
    """Cmp on the difference d under the spec cmp: ideal, f/g composite
    (d_g, d_f), Chebyshev (0, 0, D) or minimax composite (0, 0, 0, k)."""
    if isinstance(cmp, str):
        return cmp_ideal(d, 0.0)
    if is_cheb(cmp):
        return _cheb.chebval(d, cheb_step_coeffs(cmp[2]))
    if is_minimax(cmp):
        return (sign_minimax(d, cmp[3]) + 1.0) / 2.0
    return (sign_composite(d, cmp[0], cmp[1]) + 1.0) / 2.0


def comparator(cmp):
    if cmp == "ideal":
        return lambda x, y: cmp_ideal(x, y)
    return lambda x, y: cmp_of(x - y, cmp)


def embed(v, slots):
    x = np.zeros(slots)
    x[:len(v)] = v
    return x


def rank(v, N, slots, cmp="ideal"):
    """Algorithm Rank; returns the slot vector and the named intermediates."""
    x = embed(v, slots)
    VR = repl_r(x, N)
    VC = repl_c(trans_r(x, N), N)
    Cm = comparator(cmp)(VR, VC)
    S = sum_r(Cm, N)
    half = embed(np.full(N, 0.5), slots)
    R = S + half
    return R, dict(VR=VR, VC=VC, C=Cm, S=S)


def tie_offset(C, N, slots):
    """Algorithm Tie-Correction Offset from the comparison matrix C."""
    E = 4.0 * C * (1.0 - C)
    delta = np.zeros(slots)
    for i in range(N):
        for j in range(i, N):
            delta[i * N + j] = 1.0          # delta_{j >= i}: row i, column j
    U = sum_r(E * delta, N)
    T = sum_r(E, N)
    F = U - 0.5 * T - embed(np.full(N, 0.5), slots)
    return F, dict(E=E, delta=delta, U=U, T=T)


def sort(v, N, slots, cmp="ideal", ind=None):
    """Algorithm Sorting (distinct inputs).  `ind` maps a slot vector x to
    Ind_0(x); the ideal indicator is used when None."""
    x = embed(v, slots)
    R, _ = rank(v, N, slots, cmp)
    RR = repl_r(R, N)
    steps = np.zeros(slots)
    for k in range(N):
        steps[k * N:(k + 1) * N] = k + 1   # (1^N || 2^N || ... || N^N)
    D = RR - steps
    M = (np.abs(D) < 0.5).astype(float) if ind is None else ind(D)
    VR = repl_r(x, N)
    P = M * VR
    SC = sum_c(P, N)
    S = trans_c(SC, N)
    return S, dict(R=R, RR=RR, D=D, M=M, P=P, SC=SC)


def min_onehot(v, N, slots, cmp="ideal"):
    """Tie-corrected argmin: k = Rank + offset, one-hot where k = 1, value = SumC(O * V)."""
    x = embed(v, slots)
    R, inter = rank(v, N, slots, cmp)
    F, _ = tie_offset(inter["C"], N, slots)
    k = R + F
    O = np.where(np.abs(k - 1.0) < 0.5, 1.0, 0.0) * embed(np.ones(N), slots)
    val = sum_c(O * x, N)
    return O, val, k


# ---------------------------------------------------------------------------
# The circuits exactly as the CKKS code evaluates them (composite comparator,
# one-sided indicator for the minimum, merged tie-correction SumR).
# ---------------------------------------------------------------------------
def sign_composite(d, dg, df):
    """f^{d_f}(g^{d_g}(d)): the composite's odd sign approximation."""
    for _ in range(dg):
        d = poly7(d, G_COEF)
    for _ in range(df):
        d = poly7(d, F_COEF)
    return d


def argmin_circuit(v, N, slots, cmp, ind):
    """k = SumR(C + E*(delta - 1/2)) with E = C(4 - 4C) (= rank + tie offset);
    O = Cmp(1.5, k) on (1.5 - k)/N; value = SumC(O * V).  Returns (O masked to
    row 0, value slot vector, k)."""
    x = embed(v, slots)
    VR = repl_r(x, N)
    VC = repl_c(trans_r(x, N), N)
    Cm = cmp_of(VR - VC, cmp)
    E = Cm * (4.0 - 4.0 * Cm)
    tie = np.zeros(slots)
    for i in range(N):
        tie[i * N:(i + 1) * N] = np.where(np.arange(N) >= i, 0.5, -0.5)
    k = sum_r(Cm + E * tie, N)
    d = (1.5 - k) / N
    O = cmp_of(d, ind)
    val = sum_c(O * x, N)
    return mask_row(O, N, 0), val, k


def order_stat_circuit(v, N, slots, k, cmp, ind, tie):
    """Order statistic k (section 3.2), optionally tie-corrected (section 4),
    as the CKKS circuit evaluates it: the indicator is one-sided for k = 1
    (Cmp(1.5, k_j)) and k = N (Cmp(k_j, N - 1/2)) and the window
    Cmp(x, -1/2) (1 - Cmp(x, 1/2)) on x = k_j - k otherwise, every argument
    divided by N.  Without tie-correction SumR keeps no row mask (the other
    rows are annihilated by O * V).  Returns (O masked to row 0, value slot
    vector, k_j vector)."""
    x = embed(v, slots)
    VR = repl_r(x, N)
    VC = repl_c(trans_r(x, N), N)
    Cm = cmp_of(VR - VC, cmp)
    if tie:
        E = Cm * (4.0 - 4.0 * Cm)
        tm = np.zeros(slots)
        for i in range(N):
            tm[i * N:(i + 1) * N] = np.where(np.arange(N) >= i, 0.5, -0.5)
        kv = sum_r(Cm + E * tm, N)
    else:
        kv = Cm.copy()
        for i in range(log2i(N)):
            kv = kv + rot_left(kv, N << i)
        kv = kv + 0.5          # the rank
    if k == 1:
        O = cmp_of((1.5 - kv) / N, ind)
    elif k == N:
        O = cmp_of((kv - (N - 0.5)) / N, ind)
    else:
        c1 = cmp_of((kv - k + 0.5) / N, ind)
        c2 = cmp_of((kv - k - 0.5) / N, ind)
        O = c1 * (1.0 - c2)
    val = sum_c(O * x, N)
    return mask_row(O, N, 0), val, kv


def rank_multi_circuit(v, b, slots, cmp):
    """Multi-Ciphertext Ranking (section 5) on blocks of b values:
    C_{i,j} = Cmp(ReplR(B_i), ReplC(TransR(B_j))) for j >= i and
    R_i = TransC(SumC((i - 1) - sum_{j<i} C_{j,i})) + SumR(sum_{j>=i} C_{i,j}) + 1/2
    (Equation (3) for the blocks below the diagonal).  Returns [R_1..R_L]."""
    L = len(v) // b
    blocks = [embed(v[i * b:(i + 1) * b], slots) for i in range(L)]
    VR = [repl_r(x, b) for x in blocks]
    VC = [repl_c(trans_r(x, b), b) for x in blocks]
    C = {(i, j): cmp_of(VR[i] - VC[j], cmp) for i in range(L) for j in range(i, L)}
    half = embed(np.full(b, 0.5), slots)
    out = []
    for i in range(L):
        R = sum_r(sum(C[(i, j)] for j in range(i, L)), b)
        if i > 0:
            T = sum(C[(j, i)] for j in range(i))
            R = R + trans_c(sum_c(i - T, b), b)
        out.append(R + half)
    return out


def sort_multi_circuit(v, b, slots, cmp, ind):
    """Multi-Ciphertext Sorting (section 5): M_{i,j} = Ind_0(ReplR(R_j) - steps_i)
    on (x +- 1/2)/N, S_i = TransC(SumC(sum_j M_{i,j} ReplR(B_j))).  Returns [S_1..S_L]."""
    N = len(v)
    L = N // b
    R = rank_multi_circuit(v, b, slots, cmp)
    RR = [repl_r(r, b) for r in R]
    VR = [repl_r(embed(v[j * b:(j + 1) * b], slots), b) for j in range(L)]
    out = []
    for i in range(L):
        steps = np.zeros(slots)
        for r in range(b):
            steps[r * b:(r + 1) * b] = b * i + r + 1
        acc = 0.0
        for j in range(L):
            X = (RR[j] - steps) / N
            c1 = cmp_of(X + 0.5 / N, ind)
            c2 = cmp_of(X - 0.5 / N, ind)
            acc = acc + c1 * (1.0 - c2) * VR[j]
        out.append(trans_c(sum_c(acc, b), b))
    return out


def sort_circuit(v, N, slots, cmp, ind):
    """Algorithm Sorting with Ind_0(x) = Cmp(x, -1/2) (1 - Cmp(x, 1/2)) on x/N."""
    x = embed(v, slots)
    R, _ = rank(v, N, slots, cmp)
    RR = repl_r(R, N)
    steps = np.zeros(slots)
    for k in range(N):
        steps[k * N:(k + 1) * N] = k + 1
    X = RR - steps
    c1 = cmp_of((X + 0.5) / N, ind)
    c2 = cmp_of((X - 0.5) / N, ind)
    M = c1 * (1.0 - c2)
    VR = repl_r(x, N)
    SC = sum_c(M * VR, N)
    return trans_c(SC, N)


def sort_col_circuit(v, N, slots, cmp, ind):
    """Column-form Sorting (section 3.3): ranks as a column, R' = SumC(Cmp(V_C, V_R)) + 1/2;
    M = Ind_0(ReplC(R') - (1 || ... || N)^N) on (x +- 1/2)/N; S = SumR(M * ReplC(TransR(V)))."""
    x = embed(v, slots)
    VR = repl_r(x, N)
    VC = repl_c(trans_r(x, N), N)
    Cm = cmp_of(VC - VR, cmp)
    half = np.zeros(slots)
    half[0:N * N:N] = 0.5
    R = sum_c(Cm, N) + half
    RC = repl_c(R, N)
    steps = np.zeros(slots)
    for i in range(N):
        steps[i * N:(i + 1) * N] = np.arange(1, N + 1)
    X = RC - steps
    c1 = cmp_of((X + 0.5) / N, ind)
    c2 = cmp_of((X - 0.5) / N, ind)
    M = c1 * (1.0 - c2)
    return sum_r(M * VC, N)


def goldschmidt_inverse(x, iters):
    """prod_{i<iters} (1 + b^(2^i)), b = 1 - x: Goldschmidt's 1/x for x in (0, 2)"""
    b = 1.0 - x
    a = 1.0 + b
    for _ in range(1, iters):
        b = b * b
        a = a * (1.0 + b)
    return a


def order_stat_div_circuit(v, N, slots, k, cmp, ind, iters):
    """Order statistic k without tie-correction, value = SumC(O V) / SumC(O)
    (section 3.2) with the count normalised by 2 / (N + 1) and inverted by
    Goldschmidt.  Returns (mask row 0, value slot vector)."""
    O, num, _ = order_stat_circuit(v, N, slots, k, cmp, ind, False)
    s = 2.0 / (N + 1.0)
    den = sum_c(O, N)
    return O, (s * num) * goldschmidt_inverse(s * den, iters)


def rank_padded(v, slots, cmp):
    """Algorithm Rank on len(v) values that need not be a power of two
    (section 3.1): zero-padded to the next power of two Np, the comparison
    matrix masked to its N x N block before SumR."""
    N = len(v)
    Np = 1 << (N - 1).bit_length()
    x = embed(v, slots)
    VR = repl_r(x, Np)
    VC = repl_c(trans_r(x, Np), Np)
    Cm = comparator(cmp)(VR, VC)
    block = np.zeros(slots)
    for i in range(N):
        block[i * Np:i * Np + N] = 1.0
    return sum_r(Cm * block, Np) + embed(np.full(N, 0.5), slots)


def order_range_circuit(v, slots, a, b, cmp, ind, tie):
    """Mean of the order statistics a..b of the len(v) values (section 3.2,
    with the median of section 4: a = N/2, b = N/2 + 1 for even N), as the
    circuit evaluates it: the tie-corrected rank k_j (or, without
    tie-correction, the rank) in the zero-padded layout of side Np, the
    indicator Cmp(b + 1/2, k_j) when a = 1, Cmp(k_j, a - 1/2) when b = N and
    Cmp(k_j, a - 1/2) (1 - Cmp(k_j, b + 1/2)) otherwise, every argument divided
    by N; value = SumC(O x) / (b - a + 1).  Returns (O masked to the first N
    slots of row 0, value slot vector, k_j vector)."""
    N = len(v)
    Np = 1 << (N - 1).bit_length()
    x = embed(v, slots)
    VR = repl_r(x, Np)
    VC = repl_c(trans_r(x, Np), Np)
    Cm = cmp_of(VR - VC, cmp)
    if Np != N:
        block = np.zeros(slots)
        for i in range(N):
            block[i * Np:i * Np + N] = 1.0
        Cm = Cm * block
    if tie:
        E = Cm * (4.0 - 4.0 * Cm)
        tm = np.zeros(slots)
        for i in range(Np):
            tm[i * Np:(i + 1) * Np] = np.where(np.arange(Np) >= i, 0.5, -0.5)
        kv = sum_r(Cm + E * tm, Np)
    else:
        kv = Cm.copy()
        for i in range(log2i(Np)):
            kv = kv + rot_left(kv, Np << i)
        kv = kv + 0.5
    if a == 1:
        O = cmp_of((b + 0.5 - kv) / N, ind)
    elif b == N:
        O = cmp_of((kv - a + 0.5) / N, ind)
    else:
        O = cmp_of((kv - a + 0.5) / N, ind) * (1.0 - cmp_of((kv - b - 0.5) / N, ind))
    val = sum_c(O * x, Np) / (b - a + 1)
    oh = np.zeros(slots)
    oh[:N] = O[:N]
    return oh, val, kv
