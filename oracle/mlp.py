"""CPU FP64 reference of the learned block sparse approximate inverse (SPAI) of B.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).

The paper applies B^{-1} exactly (Sec. III-B: the second Krylov space needs
B^{-1} e_j).  This extension predicts the blocks of an approximate inverse M
of the overlap on B's own block pattern with a small multilayer perceptron:

  features of an atom pair (I, J), I <= J, within the pattern (F = 40):
    [0:3]   minimum-image displacement r_J - r_I divided by 4 Angstrom
    [3]     its length divided by 4 Angstrom
    [4], [5] 1 if atom I (resp. J) carries 4 orbitals
    [6:22]  10 x B_IJ, zero-padded to 4 x 4, row-major
    [22:38] 10 x (E^2)_IJ with E = B - I, zero-padded (the second-order term
            of the Neumann series of B^{-1} = sum_k (-E)^k)
    [38]    1 if I == J
    [39]    0
  network: 40 -> 128 -> 128 -> 128 -> 16, exact GELU (x Phi(x)) after each
    hidden layer, output = the 4 x 4 block M_IJ zero-padded (valid part
    n_I x n_J); M_JI = M_IJ^T; diagonal blocks symmetrised.
  parameters (flat, FP32 on the device): W1[128][40], b1[128], W2[128][128],
    b2[128], W3[128][128], b3[128], W4[16][128], b4[16]  (40,336 values).
  training target: the exact blocks (B^{-1})_IJ; loss = sum over pairs and
    valid entries of (M_IJ - target)^2 divided by the number of valid
    entries.

Everything here is plain numpy in FP64.
"""
from __future__ import annotations

import math

import numpy as np

F_IN, HID, F_OUT = 40, 128, 16
SHAPES = [(HID, F_IN), (HID,), (HID, HID), (HID,), (HID, HID), (HID,), (F_OUT, HID), (F_OUT,)]
N_PARAM = sum(int(np.prod(s)) for s in SHAPES)


def unpack(theta: np.ndarray):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def init_params(seed: int) -> np.ndarray:
    """Uniform +-sqrt(6/(fan_in+fan_out)) weights, zero biases (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            lim = math.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def pairs(sysm) -> np.ndarray:
    """Upper pairs (I <= J) of the block pattern, row-major order: int64 [n, 2]."""
    out = []
    for I in range(sysm.n_atoms):
        for b in range(sysm.blk_row_ptr[I], sysm.blk_row_ptr[I + 1]):
            J = int(sysm.blk_col[b])
            if J >= I:
                out.append((I, J))
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def _blocks(sysm, vals):
    d = {}
    for I in range(sysm.n_atoms):
        nI = int(sysm.n_orb[I])
        for b in range(sysm.blk_row_ptr[I], sysm.blk_row_ptr[I + 1]):
            J = int(sysm.blk_col[b])
            nJ = int(sysm.n_orb[J])
            d[(I, J)] = vals[sysm.val_ptr[b]:sysm.val_ptr[b + 1]].reshape(nI, nJ)
    return d


def features(sysm, P: np.ndarray) -> np.ndarray:
    """The F = 40 features of each pair (see the module docstring)."""
    Bb = _blocks(sysm, sysm.B_val)
    nb = {I: [] for I in range(sysm.n_atoms)}
    for (I, J) in Bb:
        nb[I].append(J)
    X = np.zeros((P.shape[0], F_IN))
    for p, (I, J) in enumerate(P):
        I, J = int(I), int(J)
        nI, nJ = int(sysm.n_orb[I]), int(sysm.n_orb[J])
        d = sysm.pos[J] - sysm.pos[I]
        d -= sysm.L * np.rint(d / sysm.L)
        X[p, 0:3] = d / 4.0
        X[p, 3] = np.linalg.norm(d) / 4.0
        X[p, 4] = 1.0 if nI == 4 else 0.0
        X[p, 5] = 1.0 if nJ == 4 else 0.0
        blk = np.zeros((4, 4))
        blk[:nI, :nJ] = Bb[(I, J)]
        X[p, 6:22] = 10.0 * blk.ravel()
        e2 = np.zeros((nI, nJ))
        for K in nb[I]:
            if (K, J) not in Bb:
                continue
            EIK = Bb[(I, K)] - (np.eye(nI) if K == I else 0.0)
            EKJ = Bb[(K, J)] - (np.eye(nJ) if K == J else 0.0)
            e2 += EIK @ EKJ
        blk = np.zeros((4, 4))
        blk[:nI, :nJ] = e2
        X[p, 22:38] = 10.0 * blk.ravel()
        X[p, 38] = 1.0 if I == J else 0.0
    return X


def targets(sysm, P: np.ndarray, Binv: np.ndarray):
    """Exact blocks (B^{-1})_IJ zero-padded to 4 x 4, and the valid-entry mask."""
    T = np.zeros((P.shape[0], F_OUT))
    W = np.zeros((P.shape[0], F_OUT))
    for p, (I, J) in enumerate(P):
        I, J = int(I), int(J)
        nI, nJ = int(sysm.n_orb[I]), int(sysm.n_orb[J])
        oI, oJ = int(sysm.orb_off[I]), int(sysm.orb_off[J])
        blk = np.zeros((4, 4))
        blk[:nI, :nJ] = Binv[oI:oI + nI, oJ:oJ + nJ]
        msk = np.zeros((4, 4))
        msk[:nI, :nJ] = 1.0
        T[p] = blk.ravel()
        W[p] = msk.ravel()
    return T, W


def gelu(x):
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def forward(theta, X):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    z3 = h2 @ W3.T + b3
    h3 = gelu(z3)
    out = h3 @ W4.T + b4
    return out, (X, z1, h1, z2, h2, z3, h3)


def loss_grad(theta, X, T, W):
    """Loss (masked MSE) and its gradient with respect to theta, by backpropagation."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(theta)
    out, (X, z1, h1, z2, h2, z3, h3) = forward(theta, X)
    nv = W.sum()
    r = (out - T) * W
    loss = float((r * r).sum() / nv)
    g_out = 2.0 * r / nv
    gW4 = g_out.T @ h3
    gb4 = g_out.sum(0)
    g3 = (g_out @ W4) * gelu_grad(z3)
    gW3 = g3.T @ h2
    gb3 = g3.sum(0)
    g2 = (g3 @ W3) * gelu_grad(z2)
    gW2 = g2.T @ h1
    gb2 = g2.sum(0)
    g1 = (g2 @ W2) * gelu_grad(z1)
    gW1 = g1.T @ X
    gb1 = g1.sum(0)
    grad = np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
    return loss, grad


def assemble(sysm, P: np.ndarray, out: np.ndarray) -> np.ndarray:
    """Dense M from predicted upper blocks: M_IJ, M_JI = M_IJ^T, diagonal symmetrised."""
    M = np.zeros((sysm.M, sysm.M))
    for p, (I, J) in enumerate(P):
        I, J = int(I), int(J)
        nI, nJ = int(sysm.n_orb[I]), int(sysm.n_orb[J])
        oI, oJ = int(sysm.orb_off[I]), int(sysm.orb_off[J])
        blk = out[p].reshape(4, 4)[:nI, :nJ]
        if I == J:
            blk = 0.5 * (blk + blk.T)
            M[oI:oI + nI, oI:oI + nI] = blk
        else:
            M[oI:oI + nI, oJ:oJ + nJ] = blk
            M[oJ:oJ + nJ, oI:oI + nI] = blk.T
    return M


def bf16(x):
    """Round to bfloat16 (round to nearest, ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X):
    """Inference with bfloat16 weights, inputs and hidden activations, FP64
    accumulation (the reference of a BF16 / FP32-accumulate kernel) and
    unrounded biases."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(np.asarray(theta, dtype=np.float64))
    h = bf16(X)
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        h = bf16(gelu(h @ bf16(W).T + b))
    return h @ bf16(W4).T + b4
