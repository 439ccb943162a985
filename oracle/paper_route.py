"""Second oracle route: the paper's own 3x3-mask construction (test infrastructure only).

Follows Sec. II.B-C step by step for a 3x3 mask on an N x N block, in the
paper's notation (lowercase = spatial matrices, uppercase = their DCT,
M = C.m.C^t, which is what eq. 7 gives for a = C^t.A.C):

  zero padding (Sec. II.B)
    a  row selector that moves every row down by one (first row zero),
    b  horizontal 3-tap band of mask row 1,    P = A.BLOCK.B        (eq. 6-8)
    c  horizontal 3-tap band of mask row 2,    Q = BLOCK.C_c        (eq. 9)
    d  row selector that moves every row up by one (last row zero),
    e  horizontal 3-tap band of mask row 3,    R = D.BLOCK.E        (eq. 10)
    F = P + Q + R                                                   (eq. 11)

  border replication (Sec. II.C), mask entries numbered w1..w9 row-major
    bott_cor, b_r   REPL_BOTT_COR = B_R.BLOCK.BOTT_COR               (eq. 13)
    up_cor,   u_l   REPL_UP_COR   = U_L.BLOCK.UP_COR                 (eq. 14)
    right           REPL_RIGHT    = RIGHT.BLOCK.B_R                  (eq. 15)
    left            REPL_LEFT     = LEFT.BLOCK.U_L                   (eq. 16)
    up              REPL_UP       = U_L.BLOCK.UP                     (eq. 17)
    bottom          REPL_BOTT     = B_R.BLOCK.BOTTOM                 (eq. 18)
    REPLICATION_CONDITION = sum of the six                           (eq. 19)
    F_SYMMETRICAL = F + REPLICATION_CONDITION                        (eq. 20)

The band patterns are written for any N >= 2 (the paper prints N = 8); the
printed 8 x 8 matrices are kept as a text fixture in the tests and compared
against ``spatial_matrices(W, 8)``.  The DCT matrix here is formed with numpy
from its closed form, independently of the C oracle.
"""
from __future__ import annotations

import numpy as np


def dct_matrix(N: int) -> np.ndarray:
    k = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    C = np.cos(np.pi * (2 * n + 1) * k / (2.0 * N)) * np.sqrt(2.0 / N)
    C[0, :] = np.sqrt(1.0 / N)
    return C


def _band(N: int, sub: float, diag: float, sup: float, diag_ends: bool = True) -> np.ndarray:
    """m[r][r-1] = sub, m[r][r] = diag, m[r][r+1] = sup (zero diagonal at both
    ends when ``diag_ends`` is False, as in the lateral matrices of Sec. II.C)."""
    m = np.zeros((N, N))
    for r in range(N):
        if r > 0:
            m[r, r - 1] = sub
        if r < N - 1:
            m[r, r + 1] = sup
        if diag_ends or 0 < r < N - 1:
            m[r, r] = diag
    return m


def spatial_matrices(W, N: int = 8) -> dict:
    """All spatial-domain matrices of Sec. II.B-C for the 3x3 mask ``W``."""
    W = np.asarray(W, dtype=np.float64)
    if W.shape != (3, 3):
        raise ValueError("the paper's construction is for a 3x3 mask")
    w = {f"w{p + 1}{q + 1}": W[p, q] for p in range(3) for q in range(3)}
    w1, w2, w3, w4, w5, w6, w7, w8, w9 = W.reshape(-1)
    m = {}
    # Sec. II.B: the selector a copies row i-1 into row i; b, c, e slide a
    # mask row along the columns (first column of b: w12 over w13).
    m["a"] = np.eye(N, k=-1)
    m["b"] = _band(N, sub=w["w13"], diag=w["w12"], sup=w["w11"])
    m["c"] = _band(N, sub=w["w23"], diag=w["w22"], sup=w["w21"])
    m["d"] = np.eye(N, k=1)
    m["e"] = _band(N, sub=w["w33"], diag=w["w32"], sup=w["w31"])
    # Sec. II.C: corner, separator and lateral matrices.
    m["bott_cor"] = np.zeros((N, N))
    m["bott_cor"][0, 0] = w4 + w7 + w8
    m["bott_cor"][N - 1, N - 1] = w6 + w8 + w9
    m["b_r"] = np.zeros((N, N))
    m["b_r"][N - 1, N - 1] = 1.0
    m["up_cor"] = np.zeros((N, N))
    m["up_cor"][0, 0] = w1 + w2 + w4
    m["up_cor"][N - 1, N - 1] = w2 + w3 + w6
    m["u_l"] = np.zeros((N, N))
    m["u_l"][0, 0] = 1.0
    m["up"] = _band(N, sub=w3, diag=w2, sup=w1, diag_ends=False)
    m["bottom"] = _band(N, sub=w9, diag=w8, sup=w7, diag_ends=False)
    m["right"] = _band(N, sub=w3, diag=w6, sup=w9, diag_ends=False)
    m["left"] = _band(N, sub=w1, diag=w4, sup=w7, diag_ends=False)
    return m


def dct_matrices(W, N: int = 8) -> dict:
    """Uppercase (DCT-domain) matrices M = C.m.C^t (from eq. 7)."""
    C = dct_matrix(N)
    return {k.upper(): C @ v @ C.T for k, v in spatial_matrices(W, N).items()}


def filter_zero(BLOCK, W) -> np.ndarray:
    """F = A.BLOCK.B + BLOCK.C + D.BLOCK.E (eq. 8-11)."""
    BLOCK = np.asarray(BLOCK, dtype=np.float64)
    M = dct_matrices(W, BLOCK.shape[-1])
    P = M["A"] @ BLOCK @ M["B"]
    Q = BLOCK @ M["C"]
    R = M["D"] @ BLOCK @ M["E"]
    return P + Q + R


def replication_condition(BLOCK, W) -> np.ndarray:
    """REPLICATION_CONDITION of eq. 13-19."""
    BLOCK = np.asarray(BLOCK, dtype=np.float64)
    M = dct_matrices(W, BLOCK.shape[-1])
    return (M["B_R"] @ BLOCK @ M["BOTT_COR"]
            + M["U_L"] @ BLOCK @ M["UP_COR"]
            + M["RIGHT"] @ BLOCK @ M["B_R"]
            + M["LEFT"] @ BLOCK @ M["U_L"]
            + M["U_L"] @ BLOCK @ M["UP"]
            + M["B_R"] @ BLOCK @ M["BOTTOM"])


def filter_replicate(BLOCK, W) -> np.ndarray:
    """F_SYMMETRICAL = F + REPLICATION_CONDITION (eq. 20)."""
    return filter_zero(BLOCK, W) + replication_condition(BLOCK, W)


def filter_symmetric_zero(BLOCK, W) -> np.ndarray:
    """Eq. 12 shortcut for a mask whose first and third rows agree:
    F = (A + D).BLOCK.E + BLOCK.C."""
    BLOCK = np.asarray(BLOCK, dtype=np.float64)
    M = dct_matrices(W, BLOCK.shape[-1])
    return (M["A"] + M["D"]) @ BLOCK @ M["E"] + BLOCK @ M["C"]
