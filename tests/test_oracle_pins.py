"""Pins of the FP64 oracle against facts other than itself.

Each test checks an oracle function against something the draft or
mathematics fixes independently: the draft's own 8-point butterflies and the
recursive generator of its electronic insert (evaluated here as linear maps),
forward/inverse round trips taken from separate clauses, closed forms,
library routines (matrix inverse, reflecting correlation), brute-force sums on
tiny inputs, and invariants.  None of these tests needs a GPU.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import oracle as O

DCT_FAMILY = [0, 4, 5, 6, 7, 8, 9, 10, 11]
EIGHT_CLASS = [1, 2, 3, 12, 13, 14]
# forward (I.2.3) then inverse (I.2.4) of the 8 x 8 classes: a multiple of
# the identity with this gain
EIGHT_GAIN = {1: 1.0, 2: 1.0, 3: 16.0, 12: 32.0, 13: 32.0, 14: 1.0}


# --------------------------------------------------------------------------
# The draft's 1-D transforms evaluated as linear maps
# --------------------------------------------------------------------------

def butterfly8_inverse(a):
    """I.2.1 inverse 8-point flow graph, applied to the rows of `a` (8 x m),
    arranged as an even half (inputs 0, 2, 4, 6) and an odd half (1, 3, 5, 7)
    whose outputs are added and subtracted symmetrically."""
    r2 = math.sqrt(2.0)
    c38 = math.cos(3 * math.pi / 8)
    a0, a1, a2, a3, a4, a5, a6, a7 = a
    # even half
    s04, d04 = a0 + a4, a0 - a4
    s62, d62 = a6 + a2, a6 - a2
    rot = r2 * d62 + s62
    even = [s04 + s62, d04 - rot, d04 + rot, s04 - s62]
    # odd half
    s71, d71 = a7 + a1, a7 - a1
    s53, d53 = a5 + a3, a5 - a3
    u = s71 + s53
    v = s71 - s53
    w = 2 * c38 * (d53 - d71)
    p = d71 / c38 + w
    q = 2 * r2 * c38 * d53 + w
    oa = u + p
    ob = r2 * v + oa
    odd = [u, -oa, ob, q - ob]
    out = [None] * 8
    for n in range(4):
        out[n] = even[n] + odd[n]
        out[7 - n] = even[n] - odd[n]
    return np.array(out)


def butterfly8_forward(x):
    """I.2.1 forward 8-point flow graph on the rows of `x` (8 x m), arranged
    as symmetric sums s_j = x_j + x_{7-j} (even outputs) and differences
    d_j = x_j - x_{7-j} (odd outputs)."""
    c1 = 1 / math.sqrt(2.0)
    c38 = math.cos(3 * math.pi / 8)
    s = [x[j] + x[7 - j] for j in range(4)]
    d = [x[j] - x[7 - j] for j in range(4)]
    out = [None] * 8
    out[0] = (s[0] + s[3]) + (s[1] + s[2])
    out[4] = (s[0] + s[3]) - (s[1] + s[2])
    e = c1 * ((s[1] - s[2]) + (s[0] - s[3]))
    out[2] = (s[0] - s[3]) + e
    out[6] = (s[0] - s[3]) - e
    m12 = c1 * (d[1] + d[2])
    h = c38 * ((d[2] + d[3]) - (d[0] + d[1]))
    f = (d[0] + d[1]) / (2 * c38) + h
    g = math.sqrt(2.0) * c38 * (d[2] + d[3]) + h
    out[1] = (d[0] + m12) + f
    out[7] = (d[0] + m12) - f
    out[3] = (d[0] - m12) - g
    out[5] = (d[0] - m12) + g
    return np.array(out)


class Generator:
    """The Vashkevich-Petrovsky recursion of the DCT-II/III generator insert
    (Annex R), evaluated numerically on arrays of shape (n, m) instead of
    emitting code.  N is the transform size the constants refer to."""

    def __init__(self, N):
        self.N = N

    @staticmethod
    def even_first(n):
        # the "P" permutation: even indices, then odd indices
        return list(range(0, n, 2)) + list(range(1, n, 2))

    @staticmethod
    def inverse_perm(p):
        q = [0] * len(p)
        for i, v in enumerate(p):
            q[v] = i
        return q

    @staticmethod
    def quad_order(n):
        # the "P4" permutation: index 0, then pairs taken alternately from the
        # second half and the first half, then the last first-half index
        if n <= 2:
            return list(range(n))
        half = n // 2
        seq = [0]
        top, bot, from_bottom = 1, 0, True
        while len(seq) < n - 1:
            if from_bottom:
                seq += [half + bot, half + bot + 1]
                bot += 2
            else:
                seq += [top, top + 1]
                top += 2
            from_bottom = not from_bottom
        seq.append(top)
        return seq

    def c2(self, r):
        return 2.0 * math.cos(r * math.pi / (2.0 * self.N))

    # forward
    def fwd(self, x):
        n = x.shape[0]
        if n == 1:
            return x
        h = n // 2
        top, bot = x[:h], x[h:][::-1]
        y_top, y_bot = top + bot, top - bot
        z = np.concatenate([self.fwd(y_top), self.fwd_odd(y_bot, self.N // 2)])
        out = np.empty_like(z)
        out[self.even_first(n)] = z
        return out

    def fwd_odd(self, x, r):
        n = x.shape[0]
        if n == 1:
            return x
        h = n // 2
        top, bot = x[:h], x[h:]
        t = top - bot[::-1]
        b = bot * self.c2(r)
        y = np.concatenate([t + b, t - b])
        z = np.concatenate([self.fwd_odd(y[:h], r // 2), self.fwd_odd(y[h:], self.N - r // 2)])
        return z[self.quad_order(n)]

    # inverse
    def inv(self, x):
        n = x.shape[0]
        if n == 1:
            return x
        h = n // 2
        xp = x[self.even_first(n)]
        e = self.inv(xp[:h])
        o = self.inv_odd(xp[h:], self.N // 2)
        return np.concatenate([e + o, (e - o)[::-1]])

    def inv_odd(self, x, r):
        n = x.shape[0]
        if n == 1:
            return x
        h = n // 2
        xp = x[self.inverse_perm(self.quad_order(n))]
        y = np.concatenate([self.inv_odd(xp[:h], r // 2), self.inv_odd(xp[h:], self.N - r // 2)])
        t = y[:h] + y[h:]
        b = (y[:h] - y[h:]) / self.c2(r)
        return np.concatenate([t + b[::-1], b])


def draft_inverse_matrix(N):
    if N == 8:
        return butterfly8_inverse(np.eye(8))
    return Generator(N).inv(np.eye(N))


def draft_forward_matrix(N):
    if N == 8:
        return butterfly8_forward(np.eye(8))
    return Generator(N).fwd(np.eye(N))


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_inverse_matrix_matches_draft_transform(N):
    # I.2.1 butterfly (N = 8) and the Annex R recursion (other N)
    np.testing.assert_allclose(O.idct_matrix(N), draft_inverse_matrix(N), atol=1e-12, rtol=0)


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32])
def test_forward_matrix_matches_draft_transform(N):
    np.testing.assert_allclose(O.fdct_matrix(N), draft_forward_matrix(N), atol=1e-12, rtol=0)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32])
def test_inverse_times_forward_is_N(N):
    np.testing.assert_allclose(O.idct_matrix(N) @ O.fdct_matrix(N), N * np.eye(N), atol=1e-12)


def test_generator_at_8_differs_from_butterfly_only_by_column_scale():
    # The draft uses the explicit butterfly at N = 8; the generator would give
    # the same DCT-III with other per-column scales.
    g = Generator(8).inv(np.eye(8))
    b = butterfly8_inverse(np.eye(8))
    ratio = g[0] / b[0]
    np.testing.assert_allclose(g, b * ratio[None, :], atol=1e-12)


@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 32])
def test_scale_I_makes_transform_orthonormal(N):
    # I.2.6.1: T_N diag(I(N, u)) is the orthonormal DCT-III (pins I and D).
    Q = O.idct_matrix(N) @ np.diag([O.scale_I(N, u) for u in range(N)])
    np.testing.assert_allclose(Q.T @ Q, np.eye(N), atol=1e-12)
    ref = np.array([[math.sqrt((1 if k == 0 else 2) / N) *
                     math.cos(math.pi * (2 * n + 1) * k / (2 * N)) for k in range(N)]
                    for n in range(N)])
    np.testing.assert_allclose(Q, ref, atol=1e-12)
    for u in range(N):
        assert O.scale_I(N, u) * O.scale_D(N, u) == pytest.approx(1.0 / N, rel=1e-13)


def test_scalef_reciprocal_pairs():
    # ScaleF(N, n, x) * ScaleF(n, N, x) = 1 for the pairs I.2.6 and I.2.7 use.
    for big in (8, 16, 32):
        for small in (1, 2, 4):
            for x in range(small):
                assert O.scalef(big, small, x) * O.scalef(small, big, x) == pytest.approx(1.0, rel=1e-12)


# --------------------------------------------------------------------------
# 2-D transforms per varblock type
# --------------------------------------------------------------------------

def _rng(seed=0):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("s", DCT_FAMILY)
def test_dct_family_is_direct_cosine_sum(s):
    # Brute force: every output sample as a double sum over coefficients,
    # with the 1-D maps taken from the draft's butterfly/generator.
    bx, by = O.varblock_size(s)
    K = _rng(s).standard_normal((by, bx))
    Tx, Ty = draft_inverse_matrix(bx), draft_inverse_matrix(by)
    S = O.inverse_transform(s, K)
    ref = np.zeros((by, bx))
    for n in range(by):
        for m in range(bx):
            acc = 0.0
            for k in range(by):
                for l in range(bx):
                    acc += K[k, l] * Ty[n, k] * Tx[m, l]
            ref[n, m] = acc
    np.testing.assert_allclose(S, ref, atol=1e-11)


@pytest.mark.parametrize("s,gain", [(0, 64), (4, 256), (5, 1024), (6, 128), (7, 128), (8, 256),
                                    (9, 256), (10, 512), (11, 512), (1, 1), (2, 1), (3, 16),
                                    (12, 32), (13, 32), (14, 1)])
def test_round_trip_forward_then_inverse(s, gain):
    # I.2.3 (forward) followed by I.2.4 (inverse): a multiple of the identity.
    bx, by = O.varblock_size(s)
    X = _rng(100 + s).standard_normal((by, bx))
    np.testing.assert_allclose(O.inverse_transform(s, O.forward_transform(s, X)), gain * X,
                               atol=1e-11 * gain)


@pytest.mark.parametrize("s", EIGHT_CLASS)
def test_eight_class_inverse_is_inverse_of_forward_map(s):
    # The inverse map equals numpy's inverse of the forward map (times the gain).
    gain = EIGHT_GAIN[s]
    F = np.stack([O.forward_transform(s, e.reshape(8, 8)).ravel() for e in np.eye(64)], axis=1)
    G = np.stack([O.inverse_transform(s, e.reshape(8, 8)).ravel() for e in np.eye(64)], axis=1)
    np.testing.assert_allclose(G, gain * np.linalg.inv(F), atol=1e-10)


def test_forward_of_constant_block_is_dc_only():
    for s in DCT_FAMILY + EIGHT_CLASS:
        bx, by = O.varblock_size(s)
        K = O.forward_transform(s, np.full((by, bx), 3.25))
        dc = K[0, 0]
        K[0, 0] = 0.0
        assert np.abs(K).max() < 1e-13 * abs(dc), s
        assert dc == pytest.approx(3.25 * EIGHT_GAIN.get(s, bx * by), rel=1e-12)


@pytest.mark.parametrize("s", [12, 13])
def test_half_block_transforms_are_direct_cosine_sums(s):
    # I.2.4.5 / I.2.4.6 brute force: each half is a 4 x 8 (or 8 x 4) inverse
    # built from the draft's 1-D maps, fed with every second column (row) of
    # coefficients and the DC pair combined as (0, 0) +- (1, 0) (or (0, 1));
    # DCT8x4's halves are the left and right pixel columns, DCT4x8's the top
    # and bottom pixel rows.
    K = _rng(40 + s).standard_normal((8, 8))
    S = O.inverse_transform(s, K)
    T4, T8 = draft_inverse_matrix(4), draft_inverse_matrix(8)
    ref = np.zeros((8, 8))
    for h in range(2):
        if s == 13:
            blk = K[:, h::2].copy()  # 8 rows x 4 columns
            blk[0, 0] = K[0, 0] + K[0, 1] if h == 0 else K[0, 0] - K[0, 1]
            out = np.zeros((8, 4))
            for n in range(8):
                for m in range(4):
                    out[n, m] = sum(T8[n, k] * T4[m, l] * blk[k, l] for k in range(8) for l in range(4))
            ref[:, 4 * h:4 * h + 4] = out
        else:
            blk = K[h::2, :].copy()  # 4 rows x 8 columns
            blk[0, 0] = K[0, 0] + K[1, 0] if h == 0 else K[0, 0] - K[1, 0]
            out = np.zeros((4, 8))
            for n in range(4):
                for m in range(8):
                    out[n, m] = sum(T4[n, k] * T8[m, l] * blk[k, l] for k in range(4) for l in range(8))
            ref[4 * h:4 * h + 4, :] = out
    np.testing.assert_allclose(S, ref, atol=1e-11)


def test_afv_basis_is_orthonormal():
    # The AFV basis as the oracle holds it (after the two 17-entry rows are
    # repaired): orthonormal, its first row the constant 1/4.
    B = O.afv_basis()
    np.testing.assert_allclose(B @ B.T, np.eye(16), atol=2e-14)
    np.testing.assert_allclose(B[0], np.full(16, 0.25), atol=0)


@pytest.mark.parametrize("qx,qy", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_afv_quarter_is_mirrored_basis_row(qx, qy):
    # One coefficient of one quarter (outside the 2 x 2 DC corner): the output
    # is that basis row in the quarter, mirrored horizontally for qx = 1 and
    # vertically for qy = 1, and zero elsewhere.
    B = O.afv_basis()
    for j in (3, 6, 15):
        ix, iy = j % 4, j // 4
        K = np.zeros((8, 8))
        K[qy + 2 * iy, qx + 2 * ix] = 1.0
        S = O.inverse_transform(14, K)
        q = B[j].reshape(4, 4)  # [y][x]
        if qx:
            q = q[:, ::-1]
        if qy:
            q = q[::-1, :]
        ref = np.zeros((8, 8))
        ref[4 * qy:4 * qy + 4, 4 * qx:4 * qx + 4] = q
        np.testing.assert_allclose(S, ref, atol=1e-15)


def test_identity_forward_keeps_sample_differences():
    # I.2.3.4: away from the corner slots, coefficients are differences
    # against sample (1, 1) of each 4 x 4 quarter.
    # Arrays are [row][column]: coefficient (qx + 2 ix, qy + 2 iy) of quarter
    # (qx, qy) holds sample (4 qx + ix, 4 qy + iy) minus sample (4 qx + 1, 4 qy + 1).
    X = _rng(7).standard_normal((8, 8))
    K = O.forward_transform(1, X)
    assert K[2, 1] == pytest.approx(X[1, 4] - X[1, 5])  # quarter (1, 0), (ix, iy) = (0, 1)
    assert K[5, 7] == pytest.approx(X[6, 7] - X[5, 5])  # quarter (1, 1), (ix, iy) = (3, 2)
    # the (0, 0) difference of each quarter moves to the (1, 1) slot
    assert K[3, 2] == pytest.approx(X[4, 0] - X[5, 1])  # quarter (0, 1)


# --------------------------------------------------------------------------
# LLF <-> DC (I.2.6, I.2.7)
# --------------------------------------------------------------------------

MULTI = [4, 5, 6, 7, 8, 9, 10, 11]


@pytest.mark.parametrize("s", MULTI)
def test_llf_from_dc_inverts_downsampling(s):
    bx, by = O.varblock_size(s)
    D = _rng(s).standard_normal((by // 8, bx // 8))
    np.testing.assert_allclose(O.dc_from_llf(s, O.llf_from_dc(s, D)), D, atol=1e-12)


@pytest.mark.parametrize("s", MULTI)
def test_downsampling_is_box_mean_of_lf_reconstruction(s):
    # I.2.6 equals the exact 8 x 8 means of the IDCT of the LF-only varblock.
    bx, by = O.varblock_size(s)
    cx, cy = bx // 8, by // 8
    L = _rng(30 + s).standard_normal((cy, cx))
    K = np.zeros((by, bx))
    K[:cy, :cx] = L
    S = O.inverse_transform(s, K)
    means = S.reshape(cy, 8, cx, 8).mean(axis=(1, 3))
    np.testing.assert_allclose(O.dc_from_llf(s, L), means, atol=1e-12)


def _frame_of(s, W, H, dc, ac=None, qf=1, kx=0.0, kb=0.0):
    Wb, Hb = (W + 7) // 8, (H + 7) // 8
    Wt, Ht = (W + 63) // 64, (H + 63) // 64
    return dict(ac=np.zeros((3, 8 * Hb, 8 * Wb), np.int32) if ac is None else ac,
                dc=dc.astype(np.int32), strategy=np.full((Hb, Wb), s, np.uint8),
                qf=np.full((Hb, Wb), qf - 1, np.uint8),
                sharpness=np.zeros((Hb, Wb), np.uint8),
                cfl_kx=np.full((Ht, Wt), kx, np.float32), cfl_kb=np.full((Ht, Wt), kb, np.float32))


@pytest.mark.parametrize("s", DCT_FAMILY + EIGHT_CLASS)
def test_dc_only_varblock_decodes_to_constant(s):
    bx, by = O.varblock_size(s)
    W, H = 2 * bx, 2 * by
    Wb, Hb = W // 8, H // 8
    # the same DC value in every block of a varblock, different per varblock
    vals = np.array([[5, -17], [123, -512]])
    dc = np.zeros((3, Hb, Wb))
    for c in range(3):
        dc[c] = np.kron(vals * (c + 1) // 2, np.ones((by // 8, bx // 8)))
    # DC chroma from luma (Annex G with the DC factors): X += kX_dc * Y,
    # B += kB_dc * Y, all constant per varblock.
    p = O.params(W, H, dc_mul=(0.5, 0.25, 0.125), kx_dc=0.25, kb_dc=0.875)
    xyb = O.reconstruct(p, _frame_of(s, W, H, dc))
    d = [np.kron(vals * (c + 1) // 2, np.ones((by, bx))) * p.dc_mul[c] for c in range(3)]
    np.testing.assert_allclose(xyb[1], d[1], atol=1e-12)
    np.testing.assert_allclose(xyb[0], d[0] + 0.25 * d[1], atol=1e-12)
    np.testing.assert_allclose(xyb[2], d[2] + 0.875 * d[1], atol=1e-12)


@pytest.mark.parametrize("s", DCT_FAMILY)
def test_lf_only_reconstruction_has_dc_as_block_means(s):
    bx, by = O.varblock_size(s)
    W, H = 2 * bx, 2 * by
    Wb, Hb = W // 8, H // 8
    dc = _rng(s).integers(-512, 513, size=(3, Hb, Wb))
    p = O.params(W, H, dc_mul=(1.0, 1.0, 1.0), kx_dc=0.0, kb_dc=0.0)
    xyb = O.reconstruct(p, _frame_of(s, W, H, dc))
    means = xyb.reshape(3, Hb, 8, Wb, 8).mean(axis=(2, 4))
    np.testing.assert_allclose(means, dc, atol=1e-10)


def test_cropping_keeps_top_left_samples():
    W, H = 21, 13
    dc = _rng(3).integers(-512, 513, size=(3, 2, 3))
    p = O.params(W, H, dc_mul=(1.0, 1.0, 1.0), kx_dc=0.0, kb_dc=0.0)
    xyb = O.reconstruct(p, _frame_of(0, W, H, dc))
    assert xyb.shape == (3, H, W)
    np.testing.assert_allclose(xyb[:, 8:13, 16:21], np.broadcast_to(dc[:, 1:2, 2:3], (3, 5, 5)))


# --------------------------------------------------------------------------
# Dequantization (F.3, C.6.1) and chroma from luma (Annex G)
# --------------------------------------------------------------------------

def test_dequant_matrices_positive_and_symmetric():
    for s in range(15):
        bx, by = O.varblock_size(s)
        for c in range(3):
            m = O.dequant_matrix(s, c)
            assert np.all(np.isfinite(m.ravel()[1:])) and np.all(m.ravel()[1:] > 0)
            if bx == by and s not in (12, 13, 14):
                np.testing.assert_allclose(m, m.T, rtol=1e-13)
    for a, b in [(6, 7), (8, 9), (10, 11), (12, 13)]:
        for c in range(3):
            np.testing.assert_allclose(O.dequant_matrix(a, c), O.dequant_matrix(b, c).T, rtol=1e-13)


# AFV defaults of C.6.1.1 (afv_weights per channel; the multipliers are 1)
AFV_DEFAULT = [[6368.834817724610816928, 232.1096058872860158351, 415.663547479750900044,
                220.0720486370546864556, 329.818962738766012564, -0.9919974139384578, 0, -0.60],
               [1608.323575150649711025, 67.2724358236086, 89.06657498438612, 64.07248898359674,
                125.6541247697168638611, -2.2833978673775697, -0.14, -0.2485],
               [195.927828574730424638, 21.841306388764952, 18.5279466567289584105,
                12.573868715940659, 15.89916083965558, -0.41, -0.1608, 0]]


@pytest.mark.parametrize("c", [0, 1, 2])
def test_dequant_afv_defaults(c):
    # The four low 2 x 2 cell groups hold 1 / afv_weights[0..3] (the numerators
    # are 1): group (0, 0) = the quarter DCs, (0, 1) at rows 2-3, (1, 0) at
    # columns 2-3, (1, 1); the highest frequency (kFreqs 12.97, 1e-6 below
    # the top of the printed range) takes the last band, afv_weights[4] times
    # the three band factors, to within the 1e-7 that gap makes.
    m = O.dequant_matrix(14, c)  # [y][x]
    a = AFV_DEFAULT[c]
    np.testing.assert_allclose(m[0:2, 0:2].ravel()[1:], 1.0 / a[0], rtol=1e-14)
    np.testing.assert_allclose(m[2:4, 0:2], 1.0 / a[1], rtol=1e-14)
    np.testing.assert_allclose(m[0:2, 2:4], 1.0 / a[2], rtol=1e-14)
    np.testing.assert_allclose(m[2:4, 2:4], 1.0 / a[3], rtol=1e-14)
    f = lambda v: v + 1 if v > 0 else 1 / (1 - v)
    last = a[4] * f(a[5]) * f(a[6]) * f(a[7])
    np.testing.assert_allclose(m[6:8, 6:8], 1.0 / last, rtol=3e-7)


def test_dequant_dct4x8_dc_pair_shares_the_dc_weight():
    # C.6.1 DCT4x8 mode: (x, y) takes the 8 x 4 band matrix at (x, y / 2), so
    # the second half's DC slot (0, 1) has the DC weight (multiplier 1) and
    # the DC numerator; DCT8x4 is the transpose.
    for c in range(3):
        m = O.dequant_matrix(12, c)
        assert m[1, 0] == pytest.approx(m[0, 0], rel=1e-15)
        np.testing.assert_allclose(O.dequant_matrix(13, c), m.T, rtol=1e-15)


def test_dequant_dct16_at_band_point():
    # DCT16, position (8, 8): distance sqrt(1/2), i.e. exactly band 3 of 7;
    # eccentricity 0, multiplier 1; numerator I(16, 8)^2 / 256 with
    # I(16, 8) = 1 / (16 * sqrt(2/16) * cos(pi/4)) = 1/4.
    db_y = [0.77917081615440487, -0.57424582104194355, -0.90745813428471001,
            -0.64925837484843441]
    band = db_y[0]
    for v in db_y[1:]:
        band *= (v + 1) if v > 0 else 1 / (1 - v)
    expect = (0.25 * 0.25 / 256) / band
    assert O.dequant_matrix(4, 1)[8, 8] == pytest.approx(expect, rel=1e-12)


def test_dequant_dct8_on_axis_last_band():
    # DCT8 X channel at (4, 0): distance 1/2, scaled position 5/(2 sqrt 2);
    # interpolated geometrically between bands 1 and 2; eccentricity 1 gives
    # the last eccentricity band, all factors 1.
    db = [5.0, 0.0, -0.4, -0.4, -0.4, -2.0]
    bands = [db[0]]
    for v in db[1:]:
        bands.append(bands[-1] * ((v + 1) if v > 0 else 1 / (1 - v)))
    pos = 0.5 * 5 / math.sqrt(2)
    i = int(math.floor(pos))
    w = bands[i] * (bands[i + 1] / bands[i]) ** (pos - i)
    I8 = lambda u: math.sqrt(2 / 8) * (math.sqrt(0.5) if u == 0 else 1) * math.cos(u * math.pi / 16)
    expect = I8(4) * I8(0) / 64 / w
    assert O.dequant_matrix(0, 0)[0, 4] == pytest.approx(expect, rel=1e-12)


# ---- C.6.1 encodings ------------------------------------------------------

def _flat_dct(w=(2.0, 3.0, 5.0), nb=3, ne=1):
    """A DCT-mode encoding whose weights are w[c] at every position: the
    first distance band is w[c], every later one a factor 1 (encoded 0), and
    the eccentricity bands are 1."""
    return {"mode": 6, "num_bands": nb, "num_ecc_bands": ne,
            "dist_bands": [[w[c]] + [0.0] * (nb - 1) for c in range(3)],
            "ecc_bands": [[0.0] * ne for _ in range(3)]}


def _lib15():
    return [{"mode": 0} for _ in range(15)]


def test_library_and_explicit_defaults_give_the_default_matrices():
    # Library mode stands for the C.6.1.1 encoding; that encoding written out
    # in its own mode gives the same matrices (the defaults are pinned above)
    for s in range(15):
        bx, by = O.varblock_size(s)
        explicit = _lib15()
        explicit[s] = O.default_encoding(s)
        assert explicit[s]["mode"] != 0
        for c in range(3):
            ref = O.dequant_matrix(s, c)
            np.testing.assert_array_equal(O.dequant_matrix(s, c, _lib15()), ref)
            np.testing.assert_array_equal(O.dequant_matrix(s, c, explicit), ref)


def test_copy_mode_takes_an_earlier_encoding_for_the_current_type():
    enc = _lib15()
    enc[6] = {"mode": 6, "num_bands": 4, "num_ecc_bands": 2,
              "dist_bands": [[3.0, -0.5, 0.2, -1.0]] * 3, "ecc_bands": [[0.3, -0.2]] * 3}
    enc[7] = {"mode": 7, "copy_from": 6}      # DCT8x16 copies DCT16x8's encoding
    enc[11] = {"mode": 7, "copy_from": 7}     # a copy of a copy
    enc[4] = {"mode": 7, "copy_from": 0}      # DCT16 copies DCT8, which is Library
    for c in range(3):
        # the band procedure is symmetric under exchanging the axes, and so
        # are the numerators: the copied encoding gives the transpose
        np.testing.assert_allclose(O.dequant_matrix(7, c, enc), O.dequant_matrix(6, c, enc).T,
                                   rtol=1e-14)
        # DCT16x32 evaluates DCT16x8's encoding at 16 x 32
        e11 = _lib15()
        e11[11] = dict(enc[6])
        np.testing.assert_array_equal(O.dequant_matrix(11, c, enc), O.dequant_matrix(11, c, e11))
        # DCT16 from DCT8's default encoding (DCT mode, its bands) at 16 x 16
        e4 = _lib15()
        e4[4] = O.default_encoding(0)
        np.testing.assert_array_equal(O.dequant_matrix(4, c, enc), O.dequant_matrix(4, c, e4))
        assert not np.allclose(O.dequant_matrix(4, c, enc), O.dequant_matrix(4, c))
    bad = _lib15()
    bad[5] = {"mode": 7, "copy_from": 5}      # not an earlier matrix
    with pytest.raises(O.OracleError):
        O.dequant_matrix(5, 0, bad)
    bad[5] = {"mode": 7, "copy_from": 0}
    bad[0] = {"mode": 7, "copy_from": 0}
    with pytest.raises(O.OracleError):
        O.dequant_matrix(0, 0, bad)


def test_dct_mode_two_bands_is_a_geometric_ramp():
    # two distance bands b0, b0 f(v) and one eccentricity band 1, f(e): the
    # geometric interpolation makes the weight b0 f(v)^(dist / sqrt 2)
    # f(e)^ecc, with dist = |(x / X, y / Y)| and ecc = |x / X - y / Y| / dist
    f = lambda v: v + 1 if v > 0 else 1 / (1 - v)
    for s in (0, 4, 6, 10):
        bx, by = O.varblock_size(s)
        enc = _lib15()
        enc[s] = {"mode": 6, "num_bands": 2, "num_ecc_bands": 1,
                  "dist_bands": [[2.0, -0.5], [1.5, 0.7], [0.8, -2.0]],
                  "ecc_bands": [[0.4], [-0.3], [1.1]]}
        for c in range(3):
            b0, v = enc[s]["dist_bands"][c]
            e = enc[s]["ecc_bands"][c][0]
            m = O.dequant_matrix(s, c, enc)
            x = np.arange(bx)[None, :] / bx
            y = np.arange(by)[:, None] / by
            dist = np.sqrt(x * x + y * y)
            with np.errstate(invalid="ignore", divide="ignore"):
                ecc = np.where(dist > 0, np.abs(x - y) / dist, 0.0)
            w = b0 * f(v) ** (dist / math.sqrt(2)) * f(e) ** ecc
            num = np.array([[O.scale_I(bx, i) * O.scale_I(by, j) / (bx * by) for i in range(bx)]
                            for j in range(by)])
            np.testing.assert_allclose(m.ravel()[1:], (num / w).ravel()[1:], rtol=1e-12)


@pytest.mark.parametrize("s", [0, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13])
def test_flat_weight_numerators_give_every_coefficient_the_same_energy(s):
    # C.6.1 numerators are built from I(N, u) of I.2.6.1, which makes each
    # inverse transform orthonormal once its coefficients are multiplied by
    # I: under flat weights (the same value at every position) a unit
    # quantized coefficient at any position decodes to a pixel block of the
    # same L2 energy.  The exceptions are the positions the printed steps
    # combine before the 4-point transforms: the 2 x 2 corner of DCT4 (the
    # AuxIDCT2x2 step, energy gain 4) and the DC pair of DCT4x8 / DCT8x4
    # (sum and difference, gain 2).  Swapping the axes of a non-square
    # numerator, or using the 8-point factor on a 4-point dimension, breaks
    # the equality.
    bx, by = O.varblock_size(s)
    enc = [_flat_dct() for _ in range(15)]
    for c in range(3):
        D = O.dequant_matrix(s, c, enc)
        E = np.zeros((by, bx))
        for y in range(by):
            for x in range(bx):
                K = np.zeros((by, bx))
                K[y, x] = 1.0
                E[y, x] = D[y, x] ** 2 * (O.inverse_transform(s, K) ** 2).sum()
        gain = np.ones((by, bx))
        if s == 3:
            gain[0:2, 0:2] = 4.0
        elif s == 12:
            gain[0:2, 0] = 2.0
        elif s == 13:
            gain[0, 0:2] = 2.0
        np.testing.assert_allclose(E / gain, E[-1, -1], rtol=1e-12)


def test_identity_dct2_dct4_afv_modes_place_their_parameters():
    enc = _lib15()
    idp = [[100.0, 200.0, 300.0], [10.0, 20.0, 30.0], [1.0, 2.0, 3.0]]
    d2p = [[11.0, 12.0, 13.0, 14.0, 15.0, 16.0]] * 3
    enc[1] = {"mode": 1, "params": idp}
    enc[0] = {"mode": 1, "params": idp}          # Identity mode for the DCT8 matrix
    enc[2] = {"mode": 2, "params": d2p}
    enc[3] = dict(_flat_dct(), mode=3, params=[[2.0, 4.0]] * 3)
    enc[14] = {"mode": 5, "params": [[2.0, 3.0]] * 3,
               "afv_weights": [[10.0, 20.0, 30.0, 40.0, 50.0, 0.0, 0.0, 0.0]] * 3}
    for c in range(3):
        m = O.dequant_matrix(1, c, enc)           # numerators 1
        assert m[1, 1] == 1 / idp[c][2] and m[0, 1] == m[1, 0] == 1 / idp[c][1]
        assert np.all(m[2:, :] == 1 / idp[c][0]) and np.all(m[:, 2:] == 1 / idp[c][0])
        m0 = O.dequant_matrix(0, c, enc)          # the DCT8 numerators over the same weights
        num8 = np.array([[O.scale_I(8, i) * O.scale_I(8, j) / 64 for i in range(8)] for j in range(8)])
        np.testing.assert_allclose(m0, num8 * m, rtol=1e-14)
        m = O.dequant_matrix(2, c, enc)
        np.testing.assert_array_equal(m, m.T)
        expect = {(0, 1): 11, (1, 1): 12, (2, 0): 13, (3, 1): 13, (2, 2): 14, (3, 3): 14,
                  (4, 0): 15, (7, 3): 15, (4, 4): 16, (7, 7): 16}
        for (x, y), v in expect.items():
            assert m[y, x] == 1 / v
        m = O.dequant_matrix(3, c, enc)           # flat weights 2, 3, 5 with the 2x2 corner divided
        wc = [2.0, 3.0, 5.0][c]
        num4 = np.array([[O.scale_I(4, i // 2) * O.scale_I(4, j // 2) / 64 for i in range(8)]
                         for j in range(8)])
        w = np.full((8, 8), wc)
        w[0, 1] = w[1, 0] = wc / 2.0
        w[1, 1] = wc / 4.0
        np.testing.assert_allclose(m.ravel()[1:], (num4 / w).ravel()[1:], rtol=1e-14)
        m = O.dequant_matrix(14, c, enc)
        assert np.all(m[0:2, 2:4] == 1 / 30.0) and np.all(m[2:4, 0:2] == 1 / 20.0)
        assert m[0, 1] == m[1, 0] == 1 / (10.0 * 2.0) and m[1, 1] == 1 / (10.0 * 3.0)
        assert np.all(m[2:4, 2:4] == 1 / 40.0)
        np.testing.assert_allclose(m[4:, 4:], 1 / 50.0, rtol=1e-14)   # band factors 1


def test_ill_formed_encodings_are_rejected():
    def fails(s, e):
        enc = _lib15()
        enc[s] = e
        with pytest.raises(O.OracleError):
            O.dequant_matrix(s, 0, enc)
    fails(4, {"mode": 1, "params": [[1.0, 1.0, 1.0]] * 3})     # Identity mode, 256 entries
    fails(5, {"mode": 5, "params": [[1.0, 1.0]] * 3, "afv_weights": [[1.0] * 8] * 3})
    fails(0, dict(_flat_dct(), num_bands=18))
    fails(0, dict(_flat_dct(), num_ecc_bands=0))
    fails(0, _flat_dct(w=(-1.0, -1.0, -1.0)))                 # non-positive entries
    fails(0, {"mode": 6, "num_bands": 2, "num_ecc_bands": 1,   # an infinite band
              "dist_bands": [[1.0, np.inf]] * 3, "ecc_bands": [[0.0]] * 3})
    fails(0, _flat_dct(w=(5e-324,) * 3))                      # entries overflow to inf
    fails(1, {"mode": 1, "params": [[0.0, 1.0, 1.0]] * 3})     # division by zero
    fails(0, {"mode": 8})


# ---- C.5.2 DcQuantField ---------------------------------------------------

def test_dc_smoothing_reads_each_samples_dequantization_range():
    # a 5 x 5 DC image, constant 3 but for a bump b at (2, 2); the 3x3 weights
    # sum to 1, so the average is 3 + wc b, b (1 - wc) = 0.4 below the
    # sample.  The centre is smoothed when its own field value is 1
    # (0.4 < 0.5) and kept when it is 1/2 (0.4 > 0.25); the neighbours'
    # field values do not matter
    q = O.params(40, 40, dc_mul=(1.0, 1.0, 1.0), extra_levels=(1, 1, 1), dc_smoothing=1)
    wc = 0.05226273532324128
    b = 0.4 / (1.0 - wc)
    d = np.full((3, 5, 5), 3.0)
    d[:, 2, 2] += b
    for centre, smoothed in ((1.0, True), (0.5, False)):
        fld = np.full((3, 5, 5), 0.25, np.float32)
        fld[:, 2, 2] = centre
        out = O.dc_smooth(q, d, fld)
        expect = 3.0 + wc * b if smoothed else 3.0 + b
        assert out[1, 2, 2] == pytest.approx(expect, abs=1e-12)
    # without a field: dc_mul / 2^extra_levels = 0.5, so the bump stays
    assert O.dc_smooth(q, d)[1, 2, 2] == pytest.approx(3.0 + b, abs=1e-15)


def test_qco_clamps_each_dc_sample_to_its_own_range():
    # one DCT16 varblock (2 x 2 DC samples) with an LF-only residual of 1.0
    # in each DC sample; the field allows 0.3, 0.6, 0.9 and 1.2 times 1/mul
    s = 4
    W = H = 16
    f = _qco_frame(s, W, H, qf=1)
    q = O.params(W, H, qco=1, qco_interval_mul=0.5, epf_iters=1)
    llf = O.llf_from_dc(s, np.ones((2, 2)))
    K = np.zeros((16, 16))
    K[:2, :2] = llf
    R = O.inverse_transform(s, K)
    orig = np.zeros((3, H, W))
    filt = np.repeat(R[None], 3, axis=0)
    fld = np.zeros((3, 2, 2), np.float32)
    fld[:] = np.array([[0.6, 1.2], [1.8, 2.4]], np.float32)
    f2 = dict(f, dc_quant=fld)
    out = O.qco(q, f2, orig, filt)
    for c in range(3):
        Kc = O.forward_transform(s, out[c]) / 256.0
        D = O.dc_from_llf(s, Kc[:2, :2])
        np.testing.assert_allclose(D, np.minimum(1.0, 0.5 * fld[c].astype(np.float64)), atol=1e-12)


def test_ac_prediction_window_is_the_dc_multiplier_not_the_field():
    # Annex H's 1.7 dcq window uses the channel's DC multiplier: the image
    # step is the same with extra_levels 0 and 3 and ignores the field
    rng = _rng(31)
    Hb, Wb = 6, 7
    strategy = np.zeros((Hb, Wb), np.uint8)
    d = rng.uniform(-2, 2, size=(3, Hb, Wb))
    q0 = O.params(8 * Wb, 8 * Hb, dc_mul=(1.0, 1.0, 1.0))
    q3 = O.params(8 * Wb, 8 * Hb, dc_mul=(1.0, 1.0, 1.0), extra_levels=(3, 3, 3))
    a = O.ac_prediction_image(q0, strategy, d)
    b = O.ac_prediction_image(q3, strategy, d)
    np.testing.assert_array_equal(a, b)
    fld = np.full((3, Hb, Wb), 0.01, np.float32)
    q3.dc_quant_field = fld.ctypes.data
    np.testing.assert_array_equal(O.ac_prediction_image(q3, strategy, d), a)
    q3.dc_quant_field = None


def test_field_values_must_be_positive_and_finite():
    q = O.params(16, 16)
    frame = _frame_of(0, 16, 16, np.zeros((3, 2, 2), np.int32))
    for bad in (0.0, -1.0, np.inf, np.nan):
        fld = np.ones((3, 2, 2), np.float32)
        fld[1, 1, 0] = bad
        with pytest.raises(O.OracleError):
            O.reconstruct(q, dict(frame, dc_quant=fld))


def test_ac_dequant_bias_and_cfl_linearity():
    # One DCT8 varblock with a single Y coefficient q: X gets kX times the Y
    # image, B gets kB times it (Annex G), and the Y amplitude follows the
    # F.3 bias rule.
    W = H = 8
    for q, qb in [(1, 1 - 0.07005449891748593), (-1, -(1 - 0.07005449891748593)),
                  (3, 3 - 0.145 / 3), (-5, -5 + 0.145 / 5)]:
        ac = np.zeros((3, 8, 8), np.int32)
        ac[1, 2, 3] = q
        kx, kb = 0.375, -0.625
        p = O.params(W, H, global_scale=16384, kx_dc=0.0, kb_dc=0.0)
        f = _frame_of(0, W, H, np.zeros((3, 1, 1)), ac=ac, qf=2, kx=kx, kb=kb)
        xyb = O.reconstruct(p, f)
        acmul = 65536 / (16384 * 2)
        K = np.zeros((8, 8))
        K[2, 3] = qb * acmul * O.dequant_matrix(0, 1)[2, 3]
        np.testing.assert_allclose(xyb[1], O.inverse_transform(0, K), atol=1e-14)
        np.testing.assert_allclose(xyb[0], kx * xyb[1], atol=1e-14)
        np.testing.assert_allclose(xyb[2], kb * xyb[1], atol=1e-14)


def test_ill_formed_maps_are_rejected():
    W = H = 32
    p = O.params(W, H)
    dc = np.zeros((3, 4, 4))
    f = _frame_of(0, W, H, dc)
    f["strategy"][0, 1] = 4  # DCT16 at an odd block column: not aligned
    with pytest.raises(O.OracleError):
        O.reconstruct(p, f)
    f = _frame_of(0, 24, 32, np.zeros((3, 4, 3)))
    f["strategy"][0, 0] = 5  # DCT32 needs 4 block columns, the frame has 3
    with pytest.raises(O.OracleError):
        O.reconstruct(O.params(24, 32), f)
    f = _frame_of(0, 24, 24, np.zeros((3, 3, 3)))
    f["strategy"][2, 2] = 4  # aligned but out of bounds
    with pytest.raises(O.OracleError):
        O.reconstruct(O.params(24, 24), f)
    f = _frame_of(0, W, H, dc)
    f["strategy"][0, 1] = 7  # DCT8x16 covering (1,0),(1,1)
    f["strategy"][1, 0] = 6  # DCT16x8 at (0,1) would cover (1,1) again
    with pytest.raises(O.OracleError):
        O.reconstruct(p, f)
    f = _frame_of(0, W, H, dc)
    f["strategy"][0, 0] = 15  # not a C.5.4 value
    with pytest.raises(O.OracleError):
        O.reconstruct(p, f)


# --------------------------------------------------------------------------
# Adaptive DC smoothing (F.2)
# --------------------------------------------------------------------------

# The 3x3 weights as printed (centre, edge neighbours, diagonal neighbours).
DC_SMOOTH_W = (0.05226273532324128, 0.20345139757231578, 0.0334829185968739)


def test_dc_smoothing_keeps_affine_images_and_borders():
    # the stencil is symmetric and its weights sum to one, so an affine DC
    # image is a fixed point; first/last rows and columns are never touched
    Hb, Wb = 9, 13
    y, x = np.mgrid[0:Hb, 0:Wb].astype(np.float64)
    d = np.stack([0.3 + 0.01 * x - 0.02 * y, -0.5 + 0.003 * x, 0.25 * y - 0.125 * x])
    p = O.params(8 * Wb, 8 * Hb, dc_mul=(1.0, 1.0, 1.0), dc_smoothing=1)
    out = O.dc_smooth(p, d)
    np.testing.assert_allclose(out, d, atol=1e-14)
    noisy = d + _rng(5).standard_normal(d.shape) * 0.01
    out = O.dc_smooth(p, noisy)
    np.testing.assert_array_equal(out[:, 0, :], noisy[:, 0, :])
    np.testing.assert_array_equal(out[:, -1, :], noisy[:, -1, :])
    np.testing.assert_array_equal(out[:, :, 0], noisy[:, :, 0])
    np.testing.assert_array_equal(out[:, :, -1], noisy[:, :, -1])


def test_dc_smoothing_is_the_weighted_average_when_close():
    # variations well inside 0.5 dcq: every interior sample takes the 3x3
    # weighted average (scipy's correlation with the printed weights)
    from scipy import ndimage
    wc, we, wd = DC_SMOOTH_W
    k = np.array([[wd, we, wd], [we, wc, we], [wd, we, wd]])
    d = _rng(6).standard_normal((3, 10, 12)) * 0.05
    p = O.params(96, 80, dc_mul=(2.0, 3.0, 4.0), dc_smoothing=1)
    out = O.dc_smooth(p, d)
    for c in range(3):
        ref = ndimage.correlate(d[c], k, mode="nearest")
        np.testing.assert_allclose(out[c, 1:-1, 1:-1], ref[1:-1, 1:-1], atol=1e-14)


def test_dc_smoothing_keeps_samples_far_from_the_average():
    # a checkerboard of amplitude 4 dcq: every average is far from its sample
    # (by 4 dcq (1 - wc + 4 we - 4 wd), about 6.5 dcq), so nothing changes
    y, x = np.mgrid[0:8, 0:8]
    d = np.stack([np.where((x + y) % 2 == 0, 4.0, -4.0) * q for q in (1.0, 0.5, 2.0)])
    p = O.params(64, 64, dc_mul=(1.0, 0.5, 2.0), dc_smoothing=1)
    np.testing.assert_array_equal(O.dc_smooth(p, d), d)
    # dcq follows extra_levels: dividing the multiplier by 2^levels narrows the
    # window, so a nearly flat image with a 0.3-high bump at dcq = 1 is
    # smoothed there, and left alone at dcq = 1/4
    d = np.zeros((3, 6, 6))
    d[:, 3, 3] = 0.3
    p1 = O.params(48, 48, dc_mul=(1.0, 1.0, 1.0), dc_smoothing=1)
    p4 = O.params(48, 48, dc_mul=(1.0, 1.0, 1.0), extra_levels=(2, 2, 2), dc_smoothing=1)
    assert O.dc_smooth(p1, d)[0, 3, 3] < 0.3
    assert O.dc_smooth(p4, d)[0, 3, 3] == 0.3


# --------------------------------------------------------------------------
# AC prediction (Annex H; I.2.6 / I.2.7 at N = 4)
# --------------------------------------------------------------------------

def _cell_means(S, cy4, cx4):
    return S.reshape(cy4, S.shape[0] // cy4, cx4, S.shape[1] // cx4).mean(axis=(1, 3))


@pytest.mark.parametrize("s", DCT_FAMILY + EIGHT_CLASS)
def test_dc2x2_is_cell_mean_of_lf_reconstruction(s):
    # I.2.6 at N = 4: the 4x4-pixel cell means of the varblock decoded from
    # its LLF alone (for the 8x8 types the LF reconstruction is the DC)
    bx, by = O.varblock_size(s)
    lx, ly = (bx // 8, by // 8) if s in DCT_FAMILY else (1, 1)
    L = _rng(60 + s).standard_normal((ly, lx))
    K = np.zeros((by, bx))
    K[:ly, :lx] = L
    S = O.inverse_transform(s, K)
    np.testing.assert_allclose(O.dc2x2_from_llf(s, L), _cell_means(S, 2 * ly, 2 * lx), atol=1e-12)


@pytest.mark.parametrize("s", DCT_FAMILY + EIGHT_CLASS)
def test_llf2x2_reproduces_cell_means(s):
    # I.2.7 at N = 4: the top 2cy x 2cx coefficients it gives, decoded alone,
    # have exactly the input as their 4x4-pixel cell means.  For DCT4x8 and
    # DCT8x4 this holds only with each printed form on its own type.
    bx, by = O.varblock_size(s)
    lx, ly = (bx // 8, by // 8) if s in DCT_FAMILY else (1, 1)
    cells = _rng(70 + s).standard_normal((2 * ly, 2 * lx))
    P = O.llf2x2_from_dc2x2(s, cells)
    K = np.zeros((by, bx))
    K[:2 * ly, :2 * lx] = P
    S = O.inverse_transform(s, K)
    np.testing.assert_allclose(_cell_means(S, 2 * ly, 2 * lx), cells, atol=1e-12)
    # and I.2.7 undoes I.2.6 on an LLF: the LLF back, zeros elsewhere
    L = _rng(80 + s).standard_normal((ly, lx))
    back = O.llf2x2_from_dc2x2(s, O.dc2x2_from_llf(s, L))
    np.testing.assert_allclose(back[:ly, :lx], L, atol=1e-12)
    back[:ly, :lx] = 0.0
    assert np.abs(back).max() < 1e-12


def _brute_cells(d, q):
    """Annex H image step for a frame of 8x8 types in one group, written with
    numpy / scipy: cells = the DC repeated 2x2, a border of two cells from the
    mirrored DC ring, the 3x3 average with weights 0.12 / 0.2 / 0.02 taken
    where within 1.7 q."""
    pad = np.pad(d, 1, mode="symmetric")
    img = np.kron(pad, np.ones((2, 2)))
    k = np.array([[0.02, 0.2, 0.02], [0.2, 0.12, 0.2], [0.02, 0.2, 0.02]])
    wa = ndi.correlate(img, k, mode="nearest")
    ok = np.abs(wa - img) <= 1.7 * q
    return np.where(ok, wa, img)[2:-2, 2:-2]


def test_ac_prediction_image_brute_force():
    # one group of 8x8 types with mirrored borders, against the numpy form
    Hb, Wb = 7, 11
    rng = _rng(90)
    strat = rng.choice([0, 1, 2, 3, 12, 13, 14], size=(Hb, Wb)).astype(np.uint8)
    q = (0.5, 1.0, 2.0)
    p = O.params(8 * Wb, 8 * Hb, dc_mul=q, ac_prediction=1)
    d = np.stack([rng.integers(-3, 4, size=(Hb, Wb)) * qq for qq in q]).astype(np.float64)
    got, margin = O.ac_prediction_image(p, strat, d, want_margin=True)
    k = np.array([[0.02, 0.2, 0.02], [0.2, 0.12, 0.2], [0.02, 0.2, 0.02]])
    for c in range(3):
        want = _brute_cells(d[c], q[c])
        np.testing.assert_allclose(got[c], want, atol=1e-12)
        img = np.kron(np.pad(d[c], 1, mode="symmetric"), np.ones((2, 2)))
        wa = ndi.correlate(img, k, mode="nearest")
        np.testing.assert_allclose(margin[c], (np.abs(wa - img) - 1.7 * q[c])[2:-2, 2:-2], atol=1e-12)
        assert np.abs(want - np.kron(d[c], np.ones((2, 2)))).max() > 0.1  # smoothing acted


def test_ac_prediction_groups_read_the_dc_ring():
    # two groups side by side: a DC change in the first block column of the
    # right group reaches the left group's last cells (through the ring);
    # one deeper inside does not
    Hb, Wb = 8, 64
    strat = np.zeros((Hb, Wb), np.uint8)
    p = O.params(8 * Wb, 8 * Hb, dc_mul=(1.0, 1.0, 1.0), ac_prediction=1)
    d = _rng(91).integers(-1, 2, size=(3, Hb, Wb)).astype(np.float64)
    base = O.ac_prediction_image(p, strat, d)
    d1 = d.copy()
    d1[:, 3, 32] += 1.0
    near = O.ac_prediction_image(p, strat, d1)
    assert np.abs(near[:, :, 63] - base[:, :, 63]).max() > 0.01
    d2 = d.copy()
    d2[:, 3, 40] += 1.0
    far = O.ac_prediction_image(p, strat, d2)
    np.testing.assert_array_equal(far[:, :, :64], base[:, :, :64])


@pytest.mark.parametrize("mixed", [False, True])
def test_ac_prediction_in_reconstruction(mixed):
    # frames of 8x8 types: the prediction adds, per block, coefficients whose
    # cell means are the smoothed cells minus their mean (the DC stays), so
    # the reconstruction's cell means become DC + cells - mean(cells); the
    # DC image carries the DC chroma from luma
    Hb, Wb = 6, 9
    rng = _rng(92 + mixed)
    strat = (rng.choice([0, 1, 2, 3, 12, 13, 14], size=(Hb, Wb)) if mixed
             else np.zeros((Hb, Wb))).astype(np.uint8)
    dc = rng.integers(-3, 4, size=(3, Hb, Wb))
    f = _frame_of(0, 8 * Wb, 8 * Hb, dc, kx=0.0, kb=0.0)
    f["strategy"] = strat
    kw = dict(dc_mul=(0.5, 1.0, 2.0), kx_dc=0.25, kb_dc=-0.5)
    p1 = O.params(8 * Wb, 8 * Hb, ac_prediction=1, **kw)
    p0 = O.params(8 * Wb, 8 * Hb, **kw)
    x1, x0 = O.reconstruct(p1, f), O.reconstruct(p0, f)
    assert np.abs(x1 - x0).max() > 1e-2  # the prediction is active
    dq = dc * np.array(kw["dc_mul"])[:, None, None]
    dq[0] += 0.25 * dq[1]
    dq[2] += -0.5 * dq[1]
    for c in range(3):
        q = kw["dc_mul"][c]
        cells = _brute_cells(dq[c], q)
        blockmean = np.kron(cells.reshape(Hb, 2, Wb, 2).mean(axis=(1, 3)), np.ones((2, 2)))
        want = np.kron(dq[c], np.ones((2, 2))) + cells - blockmean
        np.testing.assert_allclose(_cell_means(x1[c], 2 * Hb, 2 * Wb), want, atol=1e-10)
        np.testing.assert_allclose(_cell_means(x0[c], 2 * Hb, 2 * Wb), np.kron(dq[c], np.ones((2, 2))),
                                   atol=1e-10)


def test_ac_prediction_leaves_unsmoothed_frames_alone():
    # no cell passes the 1.7 dcq window (a DC checkerboard of amplitude 10
    # dcq) or every average equals its cell (constant DC): the prediction
    # adds nothing, whatever the types
    Hb, Wb = 8, 8
    y, x = np.mgrid[0:Hb, 0:Wb]
    strat = np.zeros((Hb, Wb), np.uint8)
    strat[0:4, 0:4] = 5
    strat[4:6, 0:2] = 4
    strat[0:4, 4:8] = np.array([[1, 2, 3, 12], [13, 14, 0, 1], [2, 3, 12, 13], [14, 0, 0, 3]])
    for dc in (np.where((x + y) % 2 == 0, 10, -10)[None].repeat(3, 0),
               np.full((3, Hb, Wb), 7)):
        f = _frame_of(0, 64, 64, dc)
        f["strategy"] = strat
        if dc.std() > 0:
            f["strategy"] = np.where(np.isin(strat, [4, 5]), 0, strat).astype(np.uint8)
        f["ac"] = _rng(93).integers(-3, 4, size=f["ac"].shape).astype(np.int32)
        kw = dict(dc_mul=(1.0, 1.0, 1.0))
        x1 = O.reconstruct(O.params(64, 64, ac_prediction=1, **kw), f)
        x0 = O.reconstruct(O.params(64, 64, **kw), f)
        np.testing.assert_allclose(x1, x0, atol=1e-9)


# --------------------------------------------------------------------------
# Quantization constraint (J.3)
# --------------------------------------------------------------------------

def _qco_frame(s, W, H, qf):
    Wb, Hb = (W + 7) // 8, (H + 7) // 8
    return dict(strategy=np.full((Hb, Wb), s, np.uint8), qf=np.asarray(qf, np.uint8))


def _corner(s):
    bx, by = O.varblock_size(s)
    return (bx // 8, by // 8) if s in DCT_FAMILY else (1, 1)


def test_qco_zero_and_small_residuals_pass_unchanged():
    # a residual whose coefficients all lie inside their intervals comes back
    # unchanged (the forward transform, scaled, is the exact inverse of the
    # inverse transform), also on a ragged frame edge
    W, H = 77, 45
    strat = _rng(1).choice([0, 1, 2, 3, 12, 13, 14], size=((H + 7) // 8, (W + 7) // 8))
    strat = strat.astype(np.uint8)
    strat[0:2, 0:2] = 4  # one DCT16 across the corner
    strat[4:6, 8:10] = 4  # and one cut by the bottom edge
    f = dict(strategy=strat, qf=_rng(2).integers(0, 256, size=strat.shape).astype(np.uint8))
    p = O.params(W, H, qco=1)
    orig = _rng(3).standard_normal((3, H, W))
    np.testing.assert_array_equal(O.qco(p, f, orig, orig), orig)
    filt = orig + 1e-9 * _rng(4).standard_normal(orig.shape)
    np.testing.assert_allclose(O.qco(p, f, orig, filt), filt, rtol=0, atol=1e-13)


@pytest.mark.parametrize("s", DCT_FAMILY + EIGHT_CLASS)
def test_qco_hf_step_is_dequant_entry_times_acmul(s):
    # one HF coefficient of amplitude A in the residual: kept below the step
    # T = qco_interval_mul * DQ * AcMul, scaled down to T above it (so the
    # whole residual is multiplied by T / A)
    bx, by = O.varblock_size(s)
    cx, cy = _corner(s)
    qf = 37
    p = O.params(bx, by, qco=1, global_scale=3, qco_interval_mul=0.75)
    acmul = 65536.0 / (3 * (1 + qf))
    f = _qco_frame(s, bx, by, np.full((by // 8, bx // 8), qf))
    orig = _rng(s).standard_normal((3, by, bx))
    for (ky, kx) in [(by - 1, bx - 1), (0, cx), (cy, 0)]:
        resid = np.zeros((3, by, bx))
        T = [0.75 * O.dequant_matrix(s, c)[ky, kx] * acmul for c in range(3)]
        for c, a in enumerate((3.0, 0.5, -2.0)):
            K = np.zeros((by, bx))
            K[ky, kx] = a * T[c]
            resid[c] = O.inverse_transform(s, K)
        out = O.qco(p, f, orig, orig + resid)
        for c, a in enumerate((3.0, 0.5, -2.0)):
            want = resid[c] * (min(abs(a), 1.0) / abs(a))
            scale = np.abs(resid[c]).max()
            np.testing.assert_allclose(out[c] - orig[c], want, atol=1e-11 * scale, err_msg=str((s, ky, kx, c)))


@pytest.mark.parametrize("s", DCT_FAMILY + EIGHT_CLASS)
def test_qco_dc_samples_clamp_to_dc_step(s):
    # a residual that is constant over each 8x8 block of the varblock's LF
    # reconstruction: its DC samples (the block means) are clamped to
    # +- qco_interval_mul * dc_mul / 2^extra_levels each, independently
    bx, by = O.varblock_size(s)
    cx, cy = _corner(s)
    p = O.params(bx, by, qco=1, dc_mul=(0.5, 2.0, 0.125), extra_levels=(1, 0, 2))
    step = [0.5 * 0.5 / 2, 0.5 * 2.0, 0.5 * 0.125 / 4]
    f = _qco_frame(s, bx, by, np.zeros((by // 8, bx // 8)))
    orig = _rng(s).standard_normal((3, by, bx))
    D = _rng(50 + s).uniform(-2.0, 2.0, size=(3, cy, cx))
    resid = np.zeros((3, by, bx))
    for c in range(3):
        K = np.zeros((by, bx))
        K[:cy, :cx] = O.llf_from_dc(s, D[c]) if (cx, cy) != (1, 1) else D[c]
        resid[c] = O.inverse_transform(s, K)
    out = O.qco(p, f, orig, orig + resid)
    for c in range(3):
        d = out[c] - orig[c]
        if (cx, cy) == (1, 1):
            # 8x8 classes: the DC is the mean of the block
            np.testing.assert_allclose(d.mean(), np.clip(D[c, 0, 0], -step[c], step[c]), atol=1e-12)
        else:
            means = d.reshape(cy, by // cy, cx, bx // cx).mean(axis=(1, 3))
            np.testing.assert_allclose(means, np.clip(D[c], -step[c], step[c]), atol=1e-12)
        # nothing but the LF part moves: the result is LF-only again
        Kout = O.forward_transform(s, d)
        Kout[:cy, :cx] = 0.0
        assert np.abs(Kout).max() < 1e-9 * max(1.0, np.abs(d).max()) * bx * by


def test_qco_is_a_projection():
    # coefficients already inside their intervals are left alone: a second
    # application changes nothing (frame of whole varblocks, so the cropped
    # samples play no part)
    W, H = 64, 64
    strat = np.zeros((8, 8), np.uint8)
    strat[0:4, 0:4] = 5
    strat[4:6, 0:2] = 4
    strat[4:5, 2:4] = 6
    strat[4:6, 4:5] = 7
    strat[6:8, 0:4] = 8
    strat[4:8, 6:8] = 11
    strat[0:4, 4:8] = np.array([[1, 2, 3, 12], [13, 14, 0, 1], [2, 3, 12, 13], [14, 0, 0, 3]])
    f = dict(strategy=strat, qf=_rng(7).integers(0, 256, size=(8, 8)).astype(np.uint8))
    p = O.params(W, H, qco=1)
    orig = _rng(8).standard_normal((3, H, W))
    filt = orig + 3.0 * _rng(9).standard_normal((3, H, W))
    once = O.qco(p, f, orig, filt)
    assert np.abs(once - filt).max() > 0.1  # the constraint is active
    np.testing.assert_allclose(O.qco(p, f, orig, once), once, atol=1e-11)


def test_qco_follows_the_filter_passes_in_decode():
    W, H = 48, 40
    Wb, Hb = 6, 5
    rng = _rng(12)
    f = _frame_of(0, W, H, rng.integers(-300, 300, size=(3, Hb, Wb)),
                  ac=rng.integers(-6, 7, size=(3, 8 * Hb, 8 * Wb)).astype(np.int32), qf=9)
    f["sharpness"] = rng.integers(0, 8, size=(Hb, Wb)).astype(np.uint8)
    base = dict(dc_mul=(0.01, 0.01, 0.01), epf_iters=2)
    pq = O.params(W, H, qco=1, **base)
    st = O.decode_stages(pq, f)
    want = O.qco(pq, f, st["recon"], st["epf"][-1][0])
    np.testing.assert_array_equal(st["qco"], want)
    np.testing.assert_allclose(O.decode(pq, f), st["rgb"], rtol=0, atol=1e-12)
    # without filter passes there is nothing to constrain
    p0q = O.params(W, H, qco=1, dc_mul=(0.01, 0.01, 0.01), epf_iters=0)
    p0 = O.params(W, H, qco=0, dc_mul=(0.01, 0.01, 0.01), epf_iters=0)
    np.testing.assert_array_equal(O.decode(p0q, f), O.decode(p0, f))
    with pytest.raises(O.OracleError):
        O.qco(O.params(W, H, qco=1, qco_interval_mul=-0.5), f, st["recon"], st["recon"])


# --------------------------------------------------------------------------
# Patches (K.3)
# --------------------------------------------------------------------------

K_CHANNEL_DEQUANT = (0.01615, 0.08875, 0.1922)  # printed in K.3


def test_patch_adds_dequantized_samples():
    W, H = 20, 12
    p = O.params(W, H)
    a = _rng(110).integers(-40, 41, size=(3, 2, 3))   # patch 0: 3 wide, 2 high
    b = _rng(111).integers(-40, 41, size=(3, 16, 16))  # patch 1: the largest size
    samples = np.concatenate([a.ravel(), b.ravel()])
    place = np.array([[4, 5, 3, 2, 0]])
    out = O.patches(p, place, samples, np.zeros((3, H, W)))
    want = np.zeros((3, H, W))
    for c in range(3):
        want[c, 5:7, 4:7] = K_CHANNEL_DEQUANT[c] * a[c]
    np.testing.assert_allclose(out, want, atol=1e-15)
    # the same patch at two overlapping places and the 16x16 one: sums
    # (a 16 x 12 patch: the frame has 12 rows)
    place = np.array([[4, 5, 3, 2, 0], [5, 6, 3, 2, 0], [4, 0, 16, 12, 18]])
    b12 = b[:, :12, :]
    samples = np.concatenate([a.ravel(), b12.ravel()])
    base = _rng(112).standard_normal((3, H, W))
    out = O.patches(p, place, samples, base)
    want = base.copy()
    for c in range(3):
        want[c, 5:7, 4:7] += K_CHANNEL_DEQUANT[c] * a[c]
        want[c, 6:8, 5:8] += K_CHANNEL_DEQUANT[c] * a[c]
        want[c, 0:12, 4:20] += K_CHANNEL_DEQUANT[c] * b12[c]
    np.testing.assert_allclose(out, want, atol=1e-13)


@pytest.mark.parametrize("bad", [[18, 0, 3, 2, 0], [0, 11, 3, 2, 0], [-1, 0, 3, 2, 0],
                                 [0, 0, 17, 1, 0], [0, 0, 0, 2, 0]])
def test_patch_outside_frame_is_ill_formed(bad):
    with pytest.raises(O.OracleError):
        O.patches(O.params(20, 12), np.array([bad]), np.zeros(3 * 17 * 2, np.int32),
                  np.zeros((3, 12, 20)))


def test_patches_precede_gaborish_in_decode():
    W, H = 40, 24
    f = _frame_of(0, W, H, _rng(113).integers(-200, 200, size=(3, 3, 5)),
                  ac=_rng(114).integers(-4, 5, size=(3, 24, 40)).astype(np.int32))
    f["patch_place"] = np.array([[3, 4, 5, 6, 0], [30, 10, 5, 6, 0]])
    f["patch_samples"] = _rng(115).integers(-20, 21, size=3 * 6 * 5)
    p = O.params(W, H, dc_mul=(0.004, 0.004, 0.004), epf_iters=1)
    st = O.decode_stages(p, f)
    np.testing.assert_array_equal(st["patches"], O.patches(p, f["patch_place"], f["patch_samples"],
                                                           st["epf"][-1][0]))
    np.testing.assert_array_equal(st["gab"], O.gaborish(p, st["patches"]))
    np.testing.assert_allclose(O.decode(p, f), st["rgb"], atol=1e-12)


# --------------------------------------------------------------------------
# Dots (K.2)
# --------------------------------------------------------------------------

def _dot(x5, y5, sx, sy, angle, sign, inten, circle):
    return [x5, y5, sx, sy, angle, sign, inten[0], inten[1], inten[2], circle]


def test_circle_dot_is_an_isotropic_gaussian():
    # a circle at (10.4, 7.2): radius = 3 / 16 (sigma + 0.5) + 0.1; every
    # sample of the 5x5 window around (10, 7) gets I exp(-d^2 / (2 r^2))
    W, H = 24, 16
    kq = (0.5, 0.25, 2.0)
    p = O.params(W, H, dot_colour_quant=kq)
    d = _dot(52, 36, 7, 7, 3, 0b010, (3, 5, 1), 1)
    out = O.dots(p, [d], np.zeros((3, H, W)))
    r = 3.0 / 16 * 7.5 + 0.1
    inten = np.array([kq[0] * 3.5, -kq[1] * 5.5, kq[2] * 1.5])
    inten[2] += 0.935669 * inten[1]
    want = np.zeros((3, H, W))
    for iy in range(5, 10):
        for ix in range(8, 13):
            g = np.exp(-((ix - 10.4) ** 2 + (iy - 7.2) ** 2) / (2 * r * r))
            want[:, iy, ix] = inten * g
    np.testing.assert_allclose(out, want, atol=1e-14)


def test_ellipse_dot_axes_and_window():
    # an ellipse of angle pi/16 (quantized 0): along its long axis the
    # Gaussian falls with sx, across with sy; a dot at the corner keeps only
    # the samples inside the frame
    W, H = 30, 20
    p = O.params(W, H, dot_colour_quant=(1.0, 1.0, 1.0))
    d = _dot(75, 50, 15, 3, 0, 0, (0, 1, 0), 0)  # centre (15, 10)
    out = O.dots(p, [d], np.zeros((3, H, W)))
    sx, sy = 3.0 / 16 * 15.5 + 0.1, 3.0 / 16 * 3.5 + 0.1
    th = np.pi / 8 * 0.5
    for iy in range(8, 13):
        for ix in range(13, 18):
            dx, dy = ix - 15, iy - 10
            along = np.cos(th) * dx + np.sin(th) * dy
            across = -np.sin(th) * dx + np.cos(th) * dy
            g = np.exp(-0.5 * (along ** 2 / sx ** 2 + across ** 2 / sy ** 2))
            assert out[1, iy, ix] == pytest.approx(1.5 * g, rel=1e-12)
    assert np.count_nonzero(out[1]) == 25
    corner = O.dots(p, [_dot(0, 0, 15, 15, 0, 0, (0, 1, 0), 1)], np.zeros((3, H, W)))
    assert np.count_nonzero(corner[1]) == 9 and corner[1, :3, :3].all()


def test_dots_follow_gaborish_and_precede_noise():
    W, H = 40, 24
    f = _frame_of(0, W, H, _rng(130).integers(-200, 200, size=(3, 3, 5)),
                  ac=_rng(131).integers(-4, 5, size=(3, 24, 40)).astype(np.int32))
    f["dots"] = np.array([_dot(60, 40, 9, 4, 5, 1, (2, 7, 3), 0), _dot(150, 90, 12, 12, 0, 4, (1, 3, 2), 1)])
    p = O.params(W, H, dc_mul=(0.004, 0.004, 0.004), epf_iters=1, noise=1,
                 noise_lut=np.full(16, 0.1), dot_colour_quant=(0.01, 0.02, 0.03))
    st = O.decode_stages(p, f)
    np.testing.assert_array_equal(st["dots"], O.dots(p, f["dots"], st["gab"]))
    np.testing.assert_array_equal(st["noise"], O.noise(p, st["dots"]))
    np.testing.assert_allclose(O.decode(p, f), st["rgb"], atol=1e-12)


# --------------------------------------------------------------------------
# Splines (K.4)
# --------------------------------------------------------------------------

def _dct_scale32(k):
    # I.2.6.1: D(32, k) = sqrt(2 / 32) eps cos(k pi / 64), eps = sqrt(1/2) at 0;
    # K.4 multiplies by 1 / (4 sqrt 2) at k = 0 and by 1/4 elsewhere
    return 1.0 / 32.0 if k == 0 else math.cos(k * math.pi / 64.0) / 16.0


def test_spline_idct_is_a_dct3_at_integer_and_quarter_points():
    import scipy.fft as sf
    c = _rng(150).standard_normal(32).astype(np.float32)
    # sum_k s_k c_k cos(k pi (t + 1/2) / 32) is scipy's unnormalized DCT-III
    # (x0 + 2 sum x_k cos(pi k (2j + 1) / 2N)) of x_0 = s_0 c_0, x_k = s_k c_k / 2
    x = np.array([_dct_scale32(k) * float(c[k]) * (1.0 if k == 0 else 0.5) for k in range(32)])
    want = sf.dct(x, type=3)
    got = [O.spline_idct(c, t) for t in range(32)]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
    # zero-padded to 64 points: t + 1/2 = (2j + 1) / 4, i.e. t = (2j - 1) / 4
    want64 = sf.dct(np.concatenate([x, np.zeros(32)]), type=3)
    got64 = [O.spline_idct(c, (2 * j - 1) / 4.0) for j in range(64)]
    np.testing.assert_allclose(got64, want64, rtol=0, atol=1e-13)
    one = np.zeros(32, np.float32)
    one[0] = 64.0
    assert O.spline_idct(one, 12.3) == pytest.approx(2.0, rel=1e-15)


def test_spline_curve_on_a_uniform_line_is_uniform():
    # collinear, equally spaced control points: the centripetal curve is the
    # line itself at a uniform parameter (every knot interval is equal)
    pts = np.array([[3, 5], [11, 11], [19, 17], [27, 23]])
    c = O.spline_curve(pts)
    assert c.shape == (16 * 3 + 1, 2)
    u = np.arange(49) / 16.0
    np.testing.assert_allclose(c, pts[0] + u[:, None] * (pts[1] - pts[0]), atol=1e-12)
    np.testing.assert_array_equal(c[::16], pts)


def _hermite_centripetal(e, n_sub=16):
    # the cubic Hermite form of one centripetal Catmull-Rom segment p1 -> p2
    # (equivalent to the Barry-Goldman pyramid the draft evaluates), with the
    # tangents of Yuksel, Schaefer and Keyser (2011)
    p0, p1, p2, p3 = (np.asarray(v, float) for v in e)
    t0 = 0.0
    t1 = t0 + np.linalg.norm(p1 - p0) ** 0.5
    t2 = t1 + np.linalg.norm(p2 - p1) ** 0.5
    t3 = t2 + np.linalg.norm(p3 - p2) ** 0.5
    m1 = (t2 - t1) * ((p1 - p0) / (t1 - t0) - (p2 - p0) / (t2 - t0) + (p2 - p1) / (t2 - t1))
    m2 = (t2 - t1) * ((p2 - p1) / (t2 - t1) - (p3 - p1) / (t3 - t1) + (p3 - p2) / (t3 - t2))
    out = []
    for k in range(n_sub):
        u = k / n_sub
        h00, h10 = 2 * u ** 3 - 3 * u ** 2 + 1, u ** 3 - 2 * u ** 2 + u
        h01, h11 = -2 * u ** 3 + 3 * u ** 2, u ** 3 - u ** 2
        out.append(h00 * p1 + h10 * m1 + h01 * p2 + h11 * m2)
    return np.array(out)


@pytest.mark.parametrize("n", [2, 3, 7])
def test_spline_curve_matches_the_hermite_form(n):
    rng = _rng(151 + n)
    pts = rng.integers(-40, 200, size=(n, 2))
    while np.any(np.all(pts[1:] == pts[:-1], axis=1)):
        pts = rng.integers(-40, 200, size=(n, 2))
    c = O.spline_curve(pts)
    e = np.concatenate([[2 * pts[0] - pts[1]], pts, [2 * pts[-1] - pts[-2]]]).astype(float)
    want = np.concatenate([_hermite_centripetal(e[w:w + 4]) for w in range(n - 1)] + [pts[-1:]])
    np.testing.assert_allclose(c, want, rtol=0, atol=1e-9)


def test_spline_curve_single_point_and_coincident_points():
    np.testing.assert_array_equal(O.spline_curve([[7, -3]]), [[7.0, -3.0]])
    assert O.spline_curve([[1, 2], [5, 6], [5, 6]]) is None


@pytest.mark.parametrize("pts", [[[0, 0], [37, 0]], [[5, 9], [30, 40], [61, 12], [80, 77]],
                                 [[0, 0], [3, 4]]])
def test_spline_walk_is_unit_arc_length_along_the_polyline(pts):
    c = O.spline_curve(pts)
    P, L = O.spline_walk(c)
    seg = np.hypot(*np.diff(c, axis=0).T)
    arc = np.concatenate([[0.0], np.cumsum(seg)])
    assert L == pytest.approx(arc[-1], rel=1e-14)
    n_int = int(math.floor(L)) + 1
    frac = L - math.floor(L)
    assert len(P) == n_int + (frac > 1e-12)
    np.testing.assert_allclose(P[:n_int, 2], np.arange(n_int))
    # positions by interpolation along the cumulative arc length
    np.testing.assert_allclose(P[:, 0], np.interp(P[:, 2], arc, c[:, 0]), atol=1e-9)
    np.testing.assert_allclose(P[:, 1], np.interp(P[:, 2], arc, c[:, 1]), atol=1e-9)
    np.testing.assert_array_equal(P[:n_int, 3], 1.0)
    if frac > 1e-12:
        np.testing.assert_allclose(P[-1], [c[-1, 0], c[-1, 1], L, frac], atol=1e-9)


def _spline_dct(values, sigma):
    # constant X, Y, B and sigma along the spline: dct[0] = 32 v
    d = np.zeros((4, 32), np.float32)
    d[:3, 0] = 32.0 * np.asarray(values)
    d[3, 0] = 32.0 * sigma
    return d


def test_spline_single_point_footprint_is_the_pixel_integral_of_a_gaussian():
    from scipy import integrate
    W, H = 40, 32
    p = O.params(W, H)
    sig, v = 2.25, (0.5, -1.0, 2.0)
    out = O.splines(p, [0, 1], [[17, 12]], _spline_dct(v, sig)[None], np.zeros((3, H, W)))
    r2 = -2.0 * sig ** 2 * math.log(0.1)
    yy, xx = np.mgrid[0:H, 0:W]
    inside = (xx - 17) ** 2 + (yy - 12) ** 2 <= r2
    np.testing.assert_array_equal(out[1] != 0, inside)
    dens = lambda y, x: math.exp(-(x * x + y * y) / (2 * sig * sig)) / (2 * math.pi * sig * sig)
    for (x, y) in [(17, 12), (19, 11), (14, 15), (20, 14)]:
        mass, _ = integrate.dblquad(dens, x - 17 - 0.5, x - 17 + 0.5, y - 12 - 0.5, y - 12 + 0.5,
                                    epsabs=1e-13)
        for c in range(3):
            assert out[c, y, x] == pytest.approx(v[c] * sig * mass, rel=1e-9)
    # the disc holds 1 - 0.1 of the continuous Gaussian's mass (pixelized)
    assert out[1].sum() == pytest.approx(-0.9 * sig, rel=0.03)


def test_spline_transposes_with_the_frame():
    W, H = 48, 36
    rng = _rng(160)
    pts = np.array([[3, 4], [20, 30], [41, 8]])
    d = rng.standard_normal((1, 4, 32)).astype(np.float32) * 0.3
    d[0, 3, 0] = 48.0  # sigma about 1.5
    a = O.splines(O.params(W, H), [0, 3], pts, d, np.zeros((3, H, W)))
    b = O.splines(O.params(H, W), [0, 3], pts[:, ::-1], d, np.zeros((3, W, H)))
    np.testing.assert_allclose(a, b.transpose(0, 2, 1), atol=1e-14)
    assert np.abs(a).max() > 0.01


def test_spline_values_follow_the_arc_length():
    # a horizontal line at integer points and a narrow sigma: pixel (x0 + j,
    # y0) sees point j alone, carrying ContinuousIDCT(31 j / L)
    W, H = 80, 16
    x0, y0, x1 = 6, 7, 66
    sig = 0.3
    d = np.zeros((1, 4, 32), np.float32)
    d[0, 0, 1] = 5.0
    d[0, 0, 3] = -2.0
    d[0, 3, 0] = 32.0 * sig
    out = O.splines(O.params(W, H), [0, 2], [[x0, y0], [x1, y0]], d, np.zeros((3, H, W)))
    L = x1 - x0
    sig = O.spline_idct(d[0, 3], 0.0)  # 0.3 rounded to binary32 via its coefficient
    g = math.erf(0.5 / (math.sqrt(2) * sig)) * 2
    for j in range(L + 1):
        want = O.spline_idct(d[0, 0], 31.0 * j / L) * sig / 4.0 * g * g
        assert out[0, y0, x0 + j] == pytest.approx(want, rel=1e-12, abs=1e-15)
    assert np.count_nonzero(out[0]) == L + 1
    # the first coefficient alone would give the same value at every pixel
    assert abs(out[0, y0, x0] - out[0, y0, x1]) > 0.01


def test_spline_points_without_positive_sigma_add_nothing():
    W, H = 40, 30
    d = _spline_dct((0.5, 1.0, -0.5), -1.5)[None]
    out = O.splines(O.params(W, H), [0, 2], [[5, 5], [30, 20]], d, np.zeros((3, H, W)))
    assert not out.any()
    d[0, 3, 0] = 0.0
    assert not O.splines(O.params(W, H), [0, 2], [[5, 5], [30, 20]], d, np.zeros((3, H, W))).any()


def test_splines_follow_dots_and_precede_noise():
    W, H = 40, 24
    f = _frame_of(0, W, H, _rng(170).integers(-200, 200, size=(3, 3, 5)),
                  ac=_rng(171).integers(-4, 5, size=(3, 24, 40)).astype(np.int32))
    f["dots"] = np.array([_dot(60, 40, 9, 4, 5, 1, (2, 7, 3), 0)])
    f["spline_offsets"] = np.array([0, 3, 4], np.int32)
    f["spline_points"] = np.array([[2, 3], [20, 15], [35, 4], [10, 18]], np.int32)
    f["spline_dct"] = np.stack([_spline_dct((0.1, 0.3, -0.2), 1.2), _spline_dct((0.0, 0.5, 0.1), 2.0)])
    p = O.params(W, H, dc_mul=(0.004, 0.004, 0.004), epf_iters=1, noise=1,
                 noise_lut=np.full(16, 0.1), dot_colour_quant=(0.01, 0.02, 0.03))
    st = O.decode_stages(p, f)
    np.testing.assert_array_equal(
        st["splines"], O.splines(p, f["spline_offsets"], f["spline_points"], f["spline_dct"],
                                 st["dots"]))
    np.testing.assert_array_equal(st["noise"], O.noise(p, st["splines"]))
    np.testing.assert_allclose(O.decode(p, f), st["rgb"], atol=1e-12)
    bad = dict(f, spline_points=np.array([[2, 3], [2, 3], [35, 4], [10, 18]], np.int32))
    with pytest.raises(O.OracleError):
        O.decode(p, bad)


# --------------------------------------------------------------------------
# JPEG1 direct rasterization (M.6)
# --------------------------------------------------------------------------

def test_jpeg1_upsampling_worked_example():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "jpeg1_upsample_example.txt")
    rows = [list(map(float, l.split())) for l in open(path) if l.strip() and not l.startswith("#")]
    np.testing.assert_array_equal(O.upsample2(rows[0]), rows[1])


def test_jpeg1_component_is_the_orthonormal_idct_of_the_dequantized_block():
    import scipy.fft as sf
    from paper_1908_03565_amd import workload as wl
    j = wl.jpeg1(40, 24, seed=190, hs=(1, 1, 1), vs=(1, 1, 1), grey=True)
    q, quant = j["coef"][0], j["quant"][0]
    pix = O.jpeg1_component(q, quant)
    for by in range(q.shape[0] // 8):
        for bx in range(q.shape[1] // 8):
            blk = q[8 * by:8 * by + 8, 8 * bx:8 * bx + 8] * quant
            # JPEG's inverse DCT: (1/4) C(u) C(v) sum ... = scipy's DCT-III, ortho
            want = sf.idctn(blk.astype(float), type=2, norm="ortho")
            np.testing.assert_allclose(pix[8 * by:8 * by + 8, 8 * bx:8 * bx + 8], want, atol=1e-10)
    # coefficient 8 u + v with u = 0, v = 1: a horizontal cosine, constant down columns
    one = np.zeros((8, 8), np.int32)
    one[0, 1] = 10
    p1 = O.jpeg1_component(one, np.ones(64, np.int32))
    assert np.ptp(p1, axis=0).max() < 1e-12 and np.ptp(p1[0]) > 1.0


def _gab_kernel(w1, w2):
    k = np.array([[w2, w1, w2], [w1, 1.0, w1], [w2, w1, w2]])
    return k / k.sum()


def test_jpeg1_gaborish_smoothing_is_the_reflecting_j4_correlation():
    # with a limit above the 36 interior pixels every block takes the
    # smoothed plane: the 3x3 kernel {1, w1, w2} normalized (J.4, the bytes
    # over 1024), mirrored at the plane's edges like scipy's "reflect"
    rng = _rng(41)
    pix = rng.uniform(-100, 100, size=(24, 40))
    code = (118, 63, 40, 255)
    out = O.jpeg1_gaborish(pix, code)
    ref = ndi.correlate(pix, _gab_kernel(118 / 1024, 63 / 1024), mode="reflect")
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)
    # limit 0: no block has fewer than 0 differing pixels, nothing changes
    np.testing.assert_array_equal(O.jpeg1_gaborish(pix, (118, 63, 40, 0)), pix)


def test_jpeg1_gaborish_counts_only_the_block_interior():
    # blocks of constant value with steps between them: the smoothing moves
    # only the pixels next to a block edge (offsets 0 and 7), which the
    # count leaves out, so with limit 1 every block is smoothed
    vals = np.array([[0.0, 50.0, -30.0], [80.0, 10.0, 20.0]])
    pix = np.kron(vals, np.ones((8, 8)))
    sm = ndi.correlate(pix, _gab_kernel(118 / 1024, 63 / 1024), mode="reflect")
    assert np.abs(sm - pix).max() > 5.0
    inner = np.zeros_like(pix, bool)
    for by in range(2):
        for bx in range(3):
            inner[8 * by + 1:8 * by + 7, 8 * bx + 1:8 * bx + 7] = True
    assert np.abs(sm - pix)[inner].max() < 1e-12
    np.testing.assert_allclose(O.jpeg1_gaborish(pix, (118, 63, 16, 1)), sm, atol=1e-12)


def test_jpeg1_gaborish_gate_brute_force():
    # random planes and codes against a direct count per block
    rng = _rng(42)
    for trial in range(12):
        hib, wib = int(rng.integers(1, 4)), int(rng.integers(1, 5))
        pix = rng.normal(0, 10, size=(8 * hib, 8 * wib))
        # some blocks get a strong pattern (many large differences)
        for by in range(hib):
            for bx in range(wib):
                if rng.random() < 0.5:
                    pix[8 * by:8 * by + 8, 8 * bx:8 * bx + 8] += 60 * (np.indices((8, 8)).sum(0) % 2)
        code = tuple(int(v) for v in (rng.integers(0, 256), rng.integers(0, 256),
                                      rng.integers(0, 256), rng.integers(0, 40)))
        sm = ndi.correlate(pix, _gab_kernel(code[0] / 1024, code[1] / 1024), mode="reflect")
        want = pix.copy()
        for by in range(hib):
            for bx in range(wib):
                d = np.abs(pix - sm)[8 * by + 1:8 * by + 7, 8 * bx + 1:8 * bx + 7]
                if (d > code[2] / 16).sum() < code[3]:
                    want[8 * by:8 * by + 8, 8 * bx:8 * bx + 8] = sm[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
        np.testing.assert_allclose(O.jpeg1_gaborish(pix, code), want, atol=1e-12)


def test_jpeg1_colour_transform_inverts_the_jfif_forward_matrix():
    # the printed constants are the JFIF forward transform's inverse to five digits
    fwd = np.array([[0.299, 0.587, 0.114], [-0.168736, -0.331264, 0.5], [0.5, -0.418688, -0.081312]])
    rng = _rng(191)
    planes = [rng.uniform(-100, 100, size=(8, 8)) for _ in range(3)]
    rgb = O.jpeg1_rasterize(planes, (1, 1, 1), (1, 1, 1), 8, 8)
    ycc = np.stack(planes).reshape(3, -1)
    want = (np.linalg.inv(fwd) @ ycc).reshape(3, 8, 8) + 128.0
    np.testing.assert_allclose(rgb, want, atol=2e-3)
    grey = O.jpeg1_rasterize(planes[:1], (1,), (1,), 8, 8)
    for c in range(3):
        np.testing.assert_allclose(grey[c], planes[0] + 128.0, atol=0)


def test_jpeg1_420_upsampling_keeps_linear_ramps_and_crops():
    # chroma planes that are linear ramps come back as linear ramps at full
    # resolution (bilinear weights) away from the mirrored edges
    Wc, Hc = 16, 8
    yy, xx = np.mgrid[0:Hc, 0:Wc]
    cb = 2.0 * xx + 0.5 * yy
    luma = np.zeros((2 * Hc, 2 * Wc))
    rgb = O.jpeg1_rasterize([luma, cb, np.zeros_like(cb)], (2, 1, 1), (2, 1, 1), 2 * Wc - 3,
                            2 * Hc - 5)
    assert rgb.shape == (3, 2 * Hc - 5, 2 * Wc - 3)
    got_cb = (rgb[2] - 128.0) / 1.772
    Y, X = np.mgrid[0:2 * Hc - 5, 0:2 * Wc - 3]
    want = 2.0 * (X - 0.5) / 2 + 0.5 * (Y - 0.5) / 2  # sample centres of the half grid
    inner = (X >= 1) & (X < 2 * Wc - 3) & (Y >= 1)
    np.testing.assert_allclose(got_cb[inner], want[inner], atol=1e-12)


# --------------------------------------------------------------------------
# Noise (K.5)
# --------------------------------------------------------------------------

M64 = 2 ** 64 - 1


def _unxorshift_right(y, k):
    # inverse of y = x ^ (x >> k) on 64 bits
    x = y
    for _ in range(64 // k + 1):
        x = y ^ (x >> k)
    return x & M64


def test_splitmix64_inverts():
    # the mixing function is a bijection; its inverse, written from the
    # printed constants (modular inverses of the odd multipliers, inverse
    # xor-shifts), undoes the oracle's value for random states
    inv1 = pow(0xBF58476D1CE4E5B9, -1, 2 ** 64)
    inv2 = pow(0x94D049BB133111EB, -1, 2 ** 64)
    rng = _rng(100)
    for z in [0, 1, M64] + [int(v) for v in rng.integers(0, 2 ** 63, size=50, dtype=np.int64)]:
        y = O.splitmix64(z)
        x = _unxorshift_right(y, 31)
        x = (x * inv2) & M64
        x = _unxorshift_right(x, 27)
        x = (x * inv1) & M64
        x = _unxorshift_right(x, 30)
        assert x == z


def test_noise_channels_are_uniform_23_bit_samples():
    ch = O.noise_channels(256, 256, 0, 0)
    assert ch.dtype == np.float32 and ch.min() >= 0.0 and ch.max() < 1.0
    m = (ch.astype(np.float64) * 2 ** 23)
    np.testing.assert_array_equal(m, np.round(m))  # exactly 23 mantissa bits
    assert np.abs(ch.mean(axis=(1, 2)) - 0.5).max() < 0.005
    assert np.abs(ch.var(axis=(1, 2)) - 1 / 12).max() < 0.002
    bits = m.astype(np.int64)
    for b in range(23):
        assert abs(((bits >> b) & 1).mean() - 0.5) < 0.01, b
    # neighbouring samples (different generators or steps) are uncorrelated
    c = ch[0].astype(np.float64) - 0.5
    assert abs((c[:, 1:] * c[:, :-1]).mean()) < 0.002
    assert abs((c[1:, :] * c[:-1, :]).mean()) < 0.002
    # deterministic per group and reseeded per group; a narrower group starts
    # with the same first segment, then its rows take fewer steps
    np.testing.assert_array_equal(O.noise_channels(256, 256, 0, 0), ch)
    other = O.noise_channels(256, 256, 256, 0)
    assert np.abs(other - ch).mean() > 0.2
    small = O.noise_channels(16, 4, 0, 0)
    np.testing.assert_array_equal(small[0, 0], ch[0, 0, :16])
    assert np.abs(small[0, 1] - ch[0, 1, :16]).max() > 0.1


# Prime factors of 2^128 - 1 = (2^64 + 1)(2^32 + 1)(2^16 + 1)(2^8 + 1)(2^4 + 1)(2^2 + 1)(2 + 1).
_ORDER_PRIMES = [3, 5, 17, 257, 641, 65537, 274177, 6700417, 67280421310721]


def _gf2_step_matrix():
    """The 128 x 128 matrix over GF(2) of one generator step, state bits
    0-63 = s0 and 64-127 = s1, built column by column from the oracle's step
    applied to the unit states (the step is linear over GF(2))."""
    M = np.zeros((128, 128), np.uint8)
    for j in range(128):
        s0, s1 = (1 << j, 0) if j < 64 else (0, 1 << (j - 64))
        _, a, b = O.noise_step(s0, s1)
        v = a | (b << 64)
        M[:, j] = [(v >> r) & 1 for r in range(128)]
    return M


def _gf2_mul(A, B):
    return (A.astype(np.float64) @ B.astype(np.float64) % 2.0).astype(np.uint8)


def _gf2_pow(sq, e):
    """M^e from the repeated squares sq[k] = M^(2^k)."""
    R = np.eye(128, dtype=np.uint8)
    k = 0
    while e:
        if e & 1:
            R = _gf2_mul(R, sq[k])
        e >>= 1
        k += 1
    return R


def test_noise_step_is_a_full_period_xorshift():
    # K.5.2 names its generator XorShift128+: a linear map of the 128-bit
    # state of maximal period, so its matrix over GF(2) has order exactly
    # 2^128 - 1.  This holds for the generator's full-period shift triple
    # and fails for a wrong shift or a step that leaves one word unchanged
    # (as the printed step taken without the exchange of the two words does).
    n = 2 ** 128 - 1
    assert math.prod(_ORDER_PRIMES) == n
    M = _gf2_step_matrix()
    # linearity: the step of a sum of states is the sum of the steps
    rng = _rng(7)
    for _ in range(4):
        a0, a1, b0, b1 = (int(v) for v in rng.integers(0, 2 ** 63, size=4, dtype=np.int64))
        _, x0, x1 = O.noise_step(a0, a1)
        _, y0, y1 = O.noise_step(b0, b1)
        _, z0, z1 = O.noise_step(a0 ^ b0, a1 ^ b1)
        assert (z0, z1) == (x0 ^ y0, x1 ^ y1)
    sq = [M]
    for _ in range(128):
        sq.append(_gf2_mul(sq[-1], sq[-1]))
    I = np.eye(128, dtype=np.uint8)
    assert np.array_equal(sq[128], M)  # M^(2^128) = M, so M^n = I
    assert np.array_equal(_gf2_pow(sq, n), I)
    for q in _ORDER_PRIMES:
        assert not np.array_equal(_gf2_pow(sq, n // q), I), q


def test_noise_step_output_is_the_sum_of_the_shifted_word_and_the_other():
    # batch[i] of K.5.2 is a sum modulo 2^64 of two words of the state, so
    # its lowest bit is linear: the xor of the two words' lowest bits (the
    # shift by 23 leaves bit 0 alone), and its carry-free low 23 bits equal
    # the xor of s0's with s1's when s0's low 23 bits are zero
    rng = _rng(8)
    for _ in range(20):
        s0, s1 = (int(v) for v in rng.integers(0, 2 ** 63, size=2, dtype=np.int64))
        b, _, _ = O.noise_step(s0, s1)
        assert (b & 1) == ((s0 ^ s1) & 1)
        b2, _, _ = O.noise_step(s0 & ~((1 << 23) - 1), s1)
        assert (b2 & ((1 << 23) - 1)) == (s1 & ((1 << 23) - 1))


def _noise_A(gw, gh, x0, y0):
    ch = O.noise_channels(gw, gh, x0, y0).astype(np.float64)
    k = np.zeros((5, 5))
    k[0, 2] = k[4, 2] = k[2, 0] = k[2, 4] = 1.0
    k[2, 2] = -4.0
    return 0.22 * np.stack([ndi.correlate(c, k, mode="reflect") for c in ch])


def test_noise_adds_lut_modulated_laplacian_of_the_channels():
    # two groups (288 x 40): LUT = k / 16, inputs spanning below 0, the LUT
    # range and above 15/14 so that the clamps act
    W, H = 288, 40
    lut = np.arange(16) / 16.0
    p = O.params(W, H, noise=1, noise_lut=lut)
    rng = _rng(101)
    xyb = np.stack([rng.uniform(-0.1, 0.1, size=(H, W)), rng.uniform(-0.2, 1.3, size=(H, W)),
                    rng.uniform(0.0, 1.0, size=(H, W))])
    out = O.noise(p, xyb)
    A = np.zeros((3, H, W))
    A[:, :, :256] = _noise_A(256, H, 0, 0)
    A[:, :, 256:] = _noise_A(32, H, 256, 0)

    def strength(v):
        # the LUT as a piecewise-linear function on [0, 15], held outside
        return np.clip(np.interp(np.clip(14.0 * v, 0.0, 15.0), np.arange(16), lut), 0.0, 1.0)

    SR, SG = strength(xyb[1] + xyb[0]), strength(xyb[1] - xyb[0])
    NR = (0.01 * A[0] + 0.99 * A[2]) * SR
    NG = (0.01 * A[1] + 0.99 * A[2]) * SG
    np.testing.assert_allclose(out[0] - xyb[0], NR - NG, atol=1e-12)
    np.testing.assert_allclose(out[1] - xyb[1], NR + NG, atol=1e-12)
    np.testing.assert_allclose(out[2] - xyb[2], 0.935669 * (NR + NG), atol=1e-12)
    inR = xyb[1] + xyb[0]
    assert np.abs(A).std() > 0.1 and (inR < 0).any() and (14 * inR >= 15).any()
    # the strength is continuous where the input crosses 0 and 15 / 14
    # (X = 0, so both inputs are Y; the same pixels just below and above)
    pn = O.params(2, 1, noise=1, noise_lut=lut)
    lo = np.zeros((3, 1, 2))
    hi = np.zeros((3, 1, 2))
    lo[1, 0] = [-1e-12, 15 / 14 - 1e-12]
    hi[1, 0] = [1e-12, 15 / 14 + 1e-12]
    np.testing.assert_allclose(O.noise(pn, lo) - lo, O.noise(pn, hi) - hi, atol=1e-9)
    # a zero LUT adds nothing
    np.testing.assert_array_equal(O.noise(O.params(W, H, noise=1), xyb), xyb)


def test_noise_follows_gaborish_in_decode():
    W, H = 40, 24
    f = _frame_of(0, W, H, _rng(102).integers(-200, 200, size=(3, 3, 5)),
                  ac=_rng(103).integers(-4, 5, size=(3, 24, 40)).astype(np.int32))
    kw = dict(dc_mul=(0.004, 0.004, 0.004), epf_iters=1, noise=1,
              noise_lut=np.linspace(0.2, 0.8, 16))
    p = O.params(W, H, **kw)
    st = O.decode_stages(p, f)
    np.testing.assert_array_equal(st["noise"], O.noise(p, st["gab"]))
    np.testing.assert_allclose(O.decode(p, f), O.xyb_to_rgb(p, st["noise"]), atol=1e-12)
    assert np.abs(st["noise"] - st["gab"]).max() > 1e-3


# --------------------------------------------------------------------------
# Gaborish (J.4)
# --------------------------------------------------------------------------

def test_gaborish_matches_reflecting_correlation():
    W, H = 19, 11
    p = O.params(W, H)
    x = _rng(5).standard_normal((3, H, W))
    out = O.gaborish(p, x)
    for c in range(3):
        w1, w2 = p.gab_w1[c], p.gab_w2[c]
        k = np.array([[w2, w1, w2], [w1, 1.0, w1], [w2, w1, w2]])
        k /= k.sum()
        np.testing.assert_allclose(out[c], ndi.correlate(x[c], k, mode="reflect"), atol=1e-13)


def test_gaborish_normalized_weights_and_constant_invariance():
    p = O.params(5, 5)
    x = np.zeros((3, 5, 5))
    x[:, 2, 2] = 1.0
    out = O.gaborish(p, x)
    norm = 1 + 4 * 0.115169525 + 4 * 0.061248592
    assert out[1, 2, 2] == pytest.approx(1 / norm, rel=1e-13)
    assert out[1, 2, 1] == pytest.approx(0.115169525 / norm, rel=1e-13)
    assert out[1, 1, 1] == pytest.approx(0.061248592 / norm, rel=1e-13)
    np.testing.assert_allclose(O.gaborish(p, np.full((3, 5, 5), 0.7)), 0.7, atol=1e-15)


# --------------------------------------------------------------------------
# Edge-preserving filter (J.2)
# --------------------------------------------------------------------------

def test_weight_closed_form_values():
    # sad = 0 gives high16 = 127 << 7, i.e. exactly 1.0 (the centre weight).
    assert O.epf_weight(0, -8128) == 1.0
    # (min(sad, 507) << 6) * mul >> 16 = -128 moves the exponent down by one.
    assert O.epf_weight(16, -8192) == 0.5
    # saturation at sad 507
    assert O.epf_weight(507, -1000) == O.epf_weight(9999, -1000)


def test_mul_table_brackets_one_half():
    t = O.mul_table(0)
    for sigma in range(16, 673, 4):
        m = t[sigma]
        assert O.epf_weight(sigma, m) > 0.5
        assert O.epf_weight(sigma, m - 1) <= 0.5
    # interpolated entries lie between their neighbours, steps truncated
    for sigma in range(16, 672, 4):
        step = int((t[sigma + 4] - t[sigma]) / 4)
        for i in range(1, 4):
            assert t[sigma + i] == t[sigma] + i * step
    assert np.all(np.diff(t[16:]) >= 0)


def _epf_frame(W, H, qf=4, sharp=7):
    Wb, Hb = (W + 7) // 8, (H + 7) // 8
    return dict(strategy=np.zeros((Hb, Wb), np.uint8), qf=np.full((Hb, Wb), qf - 1, np.uint8),
                sharpness=np.full((Hb, Wb), sharp, np.uint8))


def test_epf_constant_image_is_invariant():
    W, H = 24, 16
    p = O.params(W, H, global_scale=32768)
    x = np.stack([np.full((H, W), v) for v in (0.01, 0.4, 0.3)])
    np.testing.assert_allclose(O.epf_pass(p, _epf_frame(W, H), x), x, atol=1e-15)


def _step_case(vertical, strong):
    W = H = 32
    e = 20  # edge inside block column (or row) 2
    a = np.array([0.01, 0.30, 0.20])
    # strong: weights across the edge fall below the threshold; weak: guide
    # steps of 2, 2, 0 so that one, two and three crossed patch columns give
    # distinct surviving weights
    b = np.array([0.05, 0.80, 0.60]) if strong else np.array([0.012, 0.32, 0.21])
    x = np.empty((3, H, W))
    for c in range(3):
        if vertical:
            x[c] = np.where(np.arange(W)[None, :] >= e, b[c], a[c])
        else:
            x[c] = np.where(np.arange(H)[:, None] >= e, b[c], a[c])
    p = O.params(W, H, global_scale=32768)  # quant * quant_mul = 32768*4/65536*20 = 40
    return p, x, e, a, b


@pytest.mark.parametrize("vertical", [True, False])
@pytest.mark.parametrize("strong", [True, False])
def test_epf_step_edge_closed_form(vertical, strong):
    p, x, e, a, b = _step_case(vertical, strong)
    out, guide, sigma = O.epf_pass(p, _epf_frame(32, 32), x, want_debug=True)
    # guide bytes on both sides
    im3 = (5 * 50 / 250) ** (1 / 3)
    mins = np.array([-0.03 * im3, 0, 0])
    scale = np.array([p.epf_scale[0], p.epf_scale[1], p.epf_scale[2]])
    gl = np.floor(np.clip(((a - mins) * scale).astype(np.float32), 0, 255))
    gr = np.floor(np.clip(((b - mins) * scale).astype(np.float32), 0, 255))
    delta = int(np.abs(gl - gr).sum())
    # sigma: only the blocks holding the edge have a range, the largest
    # channel step of `scaled`; there sigma = trunc(min(range * 12.6 * 1, 40, 170))
    rng_edge = np.max(np.abs(b - a) * scale)
    sig = int(min(rng_edge * 12.6, 40.0, 170.0))
    assert sig >= 16
    for blk in range(4):
        for other in range(4):
            bxy = (other, blk) if vertical else (blk, other)
            assert sigma[bxy] == (sig if blk == 2 else 0)
    mul = O.mul_table()[sig]
    side = lambda u: u >= e
    for t in range(32):  # coordinate across the edge
        if t // 8 != 2:
            continue
        # patch extent across the edge: 4 samples horizontally, 3 vertically;
        # window offsets -3..4 horizontally, -3..3 vertically
        ext = range(-1, 3) if vertical else range(-1, 2)
        win = range(-3, 5) if vertical else range(-3, 4)
        rep = 3 if vertical else 4  # patch size along the edge
        cnt_along = 7 if vertical else 8  # window size along the edge
        wsum = np.zeros(3)
        sw = 0.0
        for o in win:
            k = sum(side(t + i) != side(t + o + i) for i in ext)
            w = O.epf_weight(rep * delta * k, mul)
            if w < 0.3:
                w = 0.0
            v = b if side(t + o) else a
            wsum += cnt_along * w * v
            sw += cnt_along * w
        expect = wsum / sw
        got = out[:, :, t].T if vertical else out[:, t, :].T
        np.testing.assert_allclose(got, np.broadcast_to(expect, (32, 3)), atol=1e-13)
    # pixels outside the edge blocks are unchanged
    mask = np.ones(32, bool)
    mask[16:24] = False
    if vertical:
        np.testing.assert_array_equal(out[:, :, mask], x[:, :, mask])
    else:
        np.testing.assert_array_equal(out[:, mask, :], x[:, mask, :])


def test_epf_guide_bytes_golden():
    # J.2.2 with the C.10 scales and target_nits_div50 = 5 (so the intensity
    # multiplier is 1): g = floor(clamp((in - min) * scale, 0, 255)),
    # min = (-0.03, 0, 0).  0.03 * 899.676941 = 26.99..., 0.28 * 899.676941 =
    # 251.90..., 1 * 111.965157, 2 * 45.275791 = 90.55...
    cases = [((0.0, 1.0, 2.0), (26, 111, 90)), ((0.25, 0.0, -0.1), (251, 0, 0)),
             ((0.3, 2.5, 6.0), (255, 255, 255)), ((-0.05, 0.5, 0.5), (0, 55, 22))]
    W, H = 8, 8
    p = O.params(W, H, global_scale=32768)
    for vals, expect in cases:
        x = np.stack([np.full((H, W), v) for v in vals])
        _, guide, _ = O.epf_pass(p, _epf_frame(W, H), x, want_debug=True)
        assert tuple(int(guide[c, 3, 3]) for c in range(3)) == expect


def test_epf_commutes_with_vertical_flip():
    W, H = 40, 32
    r = _rng(9)
    x = np.stack([0.02 * r.standard_normal((H, W)), 0.4 + 0.2 * r.standard_normal((H, W)),
                  0.3 + 0.2 * r.standard_normal((H, W))])
    f = _epf_frame(W, H)
    f["sharpness"] = r.integers(0, 8, size=f["sharpness"].shape).astype(np.uint8)
    f["qf"] = r.integers(0, 32, size=f["qf"].shape).astype(np.uint8)
    p = O.params(W, H, global_scale=32768)
    out = O.epf_pass(p, f, x)
    ff = {k: np.ascontiguousarray(v[::-1]) for k, v in f.items()}
    out_f = O.epf_pass(p, ff, np.ascontiguousarray(x[:, ::-1]))
    np.testing.assert_allclose(out_f[:, ::-1], out, atol=1e-12)
    assert np.abs(out - x).max() > 1e-3  # the filter did act


def test_epf_low_sigma_and_thresholded_weights_pass_through():
    W, H = 16, 16
    r = _rng(4)
    x = np.stack([0.02 * r.standard_normal((H, W)), 0.4 + 0.3 * r.standard_normal((H, W)),
                  0.3 + 0.3 * r.standard_normal((H, W))])
    p = O.params(W, H, global_scale=32768)
    f = _epf_frame(W, H, qf=1)  # quant * 20 = 10 < 16
    np.testing.assert_array_equal(O.epf_pass(p, f, x), x)
    f = _epf_frame(W, H, sharp=0)  # sharpness LUT entry 0
    np.testing.assert_array_equal(O.epf_pass(p, f, x), x)
    # weight 1.0 needs sad 0: with this threshold only identical patches count
    p = O.params(W, H, global_scale=32768, epf_weight_min=1.0)
    np.testing.assert_array_equal(O.epf_pass(p, _epf_frame(W, H), x), x)
    with pytest.raises(O.OracleError):  # the centre weight 1.0 must survive
        O.epf_pass(O.params(W, H, epf_weight_min=1.5), _epf_frame(W, H), x)


# --------------------------------------------------------------------------
# XYB -> RGB (L.2) and output quantization
# --------------------------------------------------------------------------

def _xyb_from_rgb(p, rgb):
    """Forward opsin transform, inverting the L.2 steps with numpy's matrix
    inverse: RGB -> mix -> gamma -> (X, Y, B)."""
    M = np.array(p.opsin_inv[:]).reshape(3, 3)
    bias = np.array(p.opsin_bias[:])
    mix = np.linalg.solve(M, rgb.reshape(3, -1)).reshape(rgb.shape)
    g = np.cbrt(mix - bias.reshape(3, 1, 1))
    return np.stack([(g[0] - g[1]) / 2, (g[0] + g[1]) / 2, g[2]])


def test_xyb_round_trip_known_colours():
    p = O.params(4, 2)
    cols = np.array([[255, 255, 255], [0, 0, 0], [128, 128, 128], [255, 0, 0],
                     [0, 255, 0], [0, 0, 255], [30, 200, 90], [250, 5, 180]], float)
    rgb = cols.T.reshape(3, 2, 4)
    xyb = _xyb_from_rgb(p, rgb)
    np.testing.assert_allclose(O.xyb_to_rgb(p, xyb), rgb / 255.0, atol=1e-12)


def test_grey_has_no_x_and_the_default_b_to_y_ratio():
    # Grey maps to X = 0, and B / Y of white is the default kB of Annex G
    # (0.935669); the opsin biases pull darker greys slightly above it.
    p = O.params(3, 1)
    rgb = np.array([[[50.0, 128.0, 255.0]]] * 3)
    xyb = _xyb_from_rgb(p, rgb)
    assert np.abs(xyb[0]).max() < 1e-6
    ratio = (xyb[2] / xyb[1]).ravel()
    assert abs(ratio[2] - 0.935669) < 5e-5
    assert np.all(np.diff(ratio) < 0) and ratio[0] - 0.935669 < 3e-4


def test_target_nits_scales_output():
    p5 = O.params(2, 1)
    p20 = O.params(2, 1, target_nits_div50=20)
    xyb = np.array([[[0.01, -0.02]], [[0.5, 0.7]], [[0.4, 0.6]]])
    np.testing.assert_allclose(O.xyb_to_rgb(p20, xyb) * 4, O.xyb_to_rgb(p5, xyb), rtol=1e-13)


@pytest.mark.parametrize("bits", [8, 16])
def test_quantize_codes_at_rounding_boundaries(bits):
    maxv = (1 << bits) - 1

    def decode(e):  # sRGB decoding function, the inverse of the encoding
        return np.where(e <= 0.04045, e / 12.92, ((e + 0.055) / 1.055) ** 2.4)

    k = np.arange(1, maxv + 1, max(1, maxv // 997))
    edge = decode((k - 0.5) / maxv)
    above = O.quantize_srgb(bits, edge * (1 + 1e-9) + 1e-15)
    below = O.quantize_srgb(bits, edge * (1 - 1e-9) - 1e-15)
    np.testing.assert_array_equal(above, k)
    np.testing.assert_array_equal(below, k - 1)
    ends = O.quantize_srgb(bits, np.array([-0.5, 0.0, 1.0, 3.0]))
    np.testing.assert_array_equal(ends, [0, 0, maxv, maxv])


def _golden_defaults():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "draft_defaults.txt")
    vals = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            name, *nums = line.split()
            vals[name] = [float(v) for v in nums]
    return vals


def test_defaults_match_draft_golden():
    # the defaults both sides start from are the values the draft prints
    # (C.10 loop filter, L.2 opsin matrix and biases, C.4.3 / Annex G factors);
    # binary32 storage allows a relative 6e-8
    from paper_1908_03565_amd import jxlr as J
    gold = _golden_defaults()
    for side, p in (("oracle", O.params(64, 64)), ("library", J.params(64, 64))):
        for name, want in gold.items():
            got = getattr(p, name)
            got = list(got) if hasattr(got, "__len__") else [got]
            np.testing.assert_allclose(got, want, rtol=6e-8, atol=0, err_msg=f"{side} {name}")
