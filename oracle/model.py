"""The functional sparse Tucker model (oracle, test infrastructure).

Eq. (1): u~(y) = sum_{j1,j2,j3} alpha_{j1 j2 j3} w1_{j1}(y1) w2_{j2}(y2) w3_{j3}(y3), and
eq. (2): w^(k)_j(y) = sum_i C_k[i, j] phi_i(y), with few non-zero C_k[i, j] (Sec. 2).  The
format is the same for any number of modes d (Sec. 2 states it for d modes); the 4-way form
carries one more factor w4_{j4}(y4) (the space-time data of Sec. 6).

Storage (Sec. 2): prod r_k core values plus the non-zero expansion coefficients; only the
values are counted, not the integers that locate them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Model:
    lo: tuple                 # box lower corner (d,)
    hi: tuple                 # box upper corner (d,)
    rank: tuple               # (r1, .., rd), d = 3 or 4
    degree: tuple             # (p1, .., pd); n_k = p_k + 1 basis functions
    core: np.ndarray          # (r1, .., rd) float64; flattened in C order j = (j1 r2 + j2) r3 + j3 ..
    coefs: list               # [C_k (n_k, r_k) float64, zeros where not in the support]
    info: dict = field(default_factory=dict)
    # per mode (s_k, q_k) of a wavelet space W_{s,q} held beside P_p (``oracle.wavelets``):
    # C_k then has p_k + 1 + (q_k + 1)(2^s_k - 1) rows; () = Legendre only
    wavelet: tuple = ()

    def mode_wavelet(self, k: int):
        return tuple(self.wavelet[k]) if self.wavelet else (0, 0)

    @property
    def R(self) -> int:
        return int(np.prod(self.rank))

    def nnz(self) -> int:
        return int(sum(np.count_nonzero(C) for C in self.coefs))

    def paper_bytes(self) -> int:
        """8 bytes per stored value: core entries plus non-zero coefficients."""
        return 8 * (self.R + self.nnz())

    def compression_ratio(self, n_points: int) -> float:
        """Original data in double precision divided by the stored values."""
        return 8.0 * n_points / self.paper_bytes()

    def with_core(self, core: np.ndarray) -> "Model":
        return Model(self.lo, self.hi, self.rank, self.degree,
                     np.asarray(core, np.float64).reshape(self.rank),
                     [C.copy() for C in self.coefs], dict(self.info), self.wavelet)


def to_csc(C: np.ndarray):
    """Compressed sparse columns (colptr, rowidx, values) of a coefficient matrix."""
    colptr = [0]
    rows, vals = [], []
    for j in range(C.shape[1]):
        nz = np.nonzero(C[:, j])[0]
        rows.extend(nz.tolist())
        vals.extend(C[nz, j].tolist())
        colptr.append(len(rows))
    return (np.asarray(colptr, np.int32), np.asarray(rows, np.int32), np.asarray(vals, np.float64))
