"""The DPP quad transpose of the fused key-switch kernel's last NTT exchange,
modelled on the host: quad_perm selector s moves to lane l the value of lane
sel(s, l) = (s >> 2l) & 3 of its quad.  The two steps (swap the off-diagonal
2 x 2 blocks with selector 0x4E, then the off-diagonal entries with 0xB1)
must transpose every quad's 4 x 4 block, which is the layout change from the
third to the fourth round of a 256-point row pass with 4 values per lane."""
import numpy as np


def _qperm(vals, sel):
    out = vals.copy()
    for lane in range(len(vals)):
        base = lane & ~3
        out[lane] = vals[base + ((sel >> (2 * (lane & 3))) & 3)]
    return out


def _quad_transpose(x):
    """x[lane][j]; the kernel's steps, lane by lane"""
    x = x.copy()
    lanes = np.arange(x.shape[0])
    l = lanes & 3
    for j in range(2):
        send = np.where(l & 2, x[:, j], x[:, j + 2])
        recv = _qperm(send, 0x4E)
        x[:, j] = np.where(l & 2, recv, x[:, j])
        x[:, j + 2] = np.where(l & 2, x[:, j + 2], recv)
    for j in (0, 2):
        send = np.where(l & 1, x[:, j], x[:, j + 1])
        recv = _qperm(send, 0xB1)
        x[:, j] = np.where(l & 1, recv, x[:, j])
        x[:, j + 1] = np.where(l & 1, x[:, j + 1], recv)
    return x


def test_selectors_are_the_xor_permutations():
    v = np.arange(8)
    assert list(_qperm(v, 0x4E)) == [2, 3, 0, 1, 6, 7, 4, 5]
    assert list(_qperm(v, 0xB1)) == [1, 0, 3, 2, 5, 4, 7, 6]


def test_round_layout_change_is_the_quad_transpose():
    """third round: lane 4h + l holds 16h + l + 4k in register k; fourth
    round: lane t holds 4t + k (rows of 256, 64 lanes)"""
    lanes = np.arange(64)
    third = np.array([[16 * (t >> 2) + (t & 3) + 4 * k for k in range(4)] for t in lanes])
    fourth = np.array([[4 * t + k for k in range(4)] for t in lanes])
    assert np.array_equal(_quad_transpose(third), fourth)
