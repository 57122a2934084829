"""Algorithmic work model of one residual evaluation, per element.

Counts follow the operations the two kernels perform (one FP64 add, multiply,
divide, square root, log or exp = 1 flop; a fused multiply-add = 2 flops); the
log means are counted on their series branch, which smooth states take almost
everywhere.  Bytes are the minimum HBM traffic of one pass: every input read
once, every output written once.
"""
from __future__ import annotations


def _sizes(dim: int, p: int):
    Q = p + 1
    NC = dim + 2
    NQ = Q ** dim
    NP = (p + 1) * (p + 2) // 2 if dim == 2 else (p + 1) * (p + 2) * (p + 3) // 6
    NQF = Q if dim == 2 else Q * Q
    NFQ = (dim + 1) * NQF
    return Q, NC, NQ, NP, NQF, NFQ


def flux_flops(dim: int, ecflux: int) -> int:
    """Directional entropy-conservative two-point flux from cached node data."""
    log_means = 13 + 13                   # {rho}_ln and 1/{rho/p}_ln
    dots = 2 * dim + 4 * 2 * dim          # {v}; {v}.n, v-.v+, v-.n, v+.n
    if ecflux == 0:                       # Ranocha
        rest = 1 + 2 + 3 * dim + 9
    else:                                 # Chandrashekar
        rest = 1 + 3 + 3 * dim + 6
    return log_means + dots + rest


def transform_macs(dim: int, p: int) -> int:
    """Multiply-adds of one sum-factorised application of V (or V^T) to one variable."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    if dim == 2:
        return NP * Q + (p + 1) * Q * Q
    npair = (p + 1) * (p + 2) // 2
    return NP * Q + npair * Q * Q + (p + 1) * Q ** 3


def pair_counts(dim: int, p: int):
    """(volume pairs with two direction terms, with one, facet-correction pairs,
    interface nodes) per element, evaluated once each by the line loops."""
    Q = p + 1
    per_line = Q * (Q - 1) // 2
    lines = Q ** (dim - 1)
    if dim == 2:
        return lines * per_line, lines * per_line, 3 * Q * Q, 3 * Q
    return 2 * lines * per_line, lines * per_line, 3 * Q ** 3 + Q ** 4, 4 * Q * Q


def k2_flops(dim: int, p: int, ecflux: int = 0, dissipation: int = 1) -> int:
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    F = flux_flops(dim, ecflux)
    v2, v1, fc, nif = pair_counts(dim, p)
    conv = 3 * dim + 9                                        # U(w) per node
    vol = v2 * (F + 5 * dim + 2 * NC) + v1 * (F + 2 * dim + 2 * NC)
    fac = fc * (F + 2 * dim + NC + 2 * NC)
    diss = (11 * dim + 21 + 2 * NC) if dissipation else 0
    iface = nif * (conv + F + diss + 2 * NC)
    xf = 4 * NC * 2 * transform_macs(dim, p) + NC * NQ        # V, V^T, V, V^T and w/J
    rt = NC * NQ * (8 if dim == 3 else 6) + (NC * Q ** 3 * 2 if dim == 3 else 0)
    return vol + fac + iface + xf + rt + (NQ + NFQ) * conv


def k1_flops(dim: int, p: int) -> int:
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    wvars = NQ * (7 * dim + 14 + NC)                           # W(u) times w J
    xf = 5 * NC * 2 * transform_macs(dim, p) + NC * NQ
    ext = NC * (2 * 5 * Q ** 3 if dim == 3 else 2 * 3 * Q * Q)
    return wvars + xf + ext


def k2_bytes(dim: int, p: int) -> int:
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    ngv = 8 if dim == 2 else 17
    return 8 * (NC * NP + 2 * NC * NFQ + (ngv - 1) * NQ + (dim + 1) * NFQ + NC * NP) + 4 * NFQ


def k2_rk_bytes(dim: int, p: int) -> int:
    """K2 inside an RK4 step with the stage combination formed by its output:
    instead of writing du~/dt it reads u and acc and writes acc and U (stage 1
    skips the acc read, stage 4 reads acc and writes u), 3.25 state arrays on
    average over the four stages in place of one."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    return k2_bytes(dim, p) + (8 * NC * NP * 9) // 4


def k2_next_bytes(dim: int, p: int) -> int:
    """The RK4 stage kernel: K2 whose output is the stage combination and which
    then projects the next stage input of its elements (K1's work on data
    already in LDS).  Against the plain residual it moves, per element, 2.5
    state arrays on average over the four stages instead of du~/dt (stage 1:
    u read, acc written; stages 2-3: u and acc read, acc written; stage 4: acc
    read, u written), plus the projection's w J read and w~ and facet values
    written."""
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    return k2_bytes(dim, p) + (8 * NC * NP * 3) // 2 + 8 * (NC * NP + NC * NFQ + NQ)


def k1_bytes(dim: int, p: int) -> int:
    Q, NC, NQ, NP, NQF, NFQ = _sizes(dim, p)
    return 8 * (NC * NP + 2 * NQ + NC * NP + NC * NFQ)


PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 vector
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
