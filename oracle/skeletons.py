"""Block Arnoldi skeletons (oracle, FP64).

Test infrastructure only: see the package docstring.

Each skeleton builds, for one restart cycle, the block basis V_1, V_2, ...
(n x s blocks) and the block upper Hessenberg matrix H of the block Arnoldi
relation A V_j = V_{j+1} H_{1:j+1,1:j} (Sec. 2.4, eq. block_arnoldi), one
block column at a time.  ``run(R0)`` is a generator that yields j each time
block column j of H is final (including its subdiagonal block H_{j+1,j}) and
V_{j+1} exists.  The driver may stop it after any column.

Indices in comments are the paper's (1-based blocks); arrays are 0-based.

Counters follow Sec. 2.1 and Sec. 5: an A-call is one product with A; a sync
is one block inner product or one IntraOrtho call (Sec. 2.3).  Applications
of the basis are counted as the per-cycle totals printed in the appendix
tables imply: a fused inner product whose left factor is [V X] counts two, a
block inner product or a projection/update with the basis counts one.

A Cholesky breakdown (the NaN-flag of Sec. 4) stops the cycle; ``flagged`` is
then set and ``last`` holds the last block column that is final.  Reading:
in the delayed skeletons (Algs. 6 and 7) the Cholesky at loop step k yields
H_{k,k-1}, so a flag there leaves k-2 final columns; in Algs. 2, 3 and 5 the
factor at step k is H_{k+1,k}, leaving k-1.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .primitives import (chol_flag, intra_ortho, ip, ip_global, left_solve_upper_t, muscle_syncs,
                         right_solve_upper)


class Counters:
    def __init__(self):
        self.a_calls = 0
        self.v_apps = 0
        self.syncs = 0

    def as_tuple(self):
        return (self.a_calls, self.v_apps, self.syncs)


class _Skeleton:
    delayed = False

    def __init__(self, A, s: int, m: int, muscle: str, counters: Counters, force_steps=()):
        self.A = A
        self.s = s
        self.m = m
        self.muscle = muscle
        self.ct = counters
        self.force_steps = set(force_steps)   # loop steps k whose Cholesky is forced to flag
        self.V: list[np.ndarray] = []
        self.flagged = False
        self.last = 0
        self.Beta = None
        # room for the column m+1 that the delayed skeletons touch at their last step
        self.H = np.zeros(((m + 2) * s, (m + 1) * s))

    # -- helpers -------------------------------------------------------------------
    def blk(self, i: int) -> slice:
        """Rows/cols of 1-based block i."""
        return slice((i - 1) * self.s, i * self.s)

    def upto(self, i: int) -> slice:
        """Rows/cols of blocks 1..i."""
        return slice(0, i * self.s)

    def Vcat(self, i: int) -> np.ndarray:
        """[V_1 ... V_i] as an n x is array."""
        return np.hstack(self.V[:i])

    def ip(self, X, Y):
        """The block inner product of the paradigm (Sec. 2.2, Table 1):
        classical X^T Y, or the global one when the muscle is "global"."""
        if self.muscle == "global":
            return ip_global(X, Y, self.s)
        return ip(X, Y)

    def matvec(self, X):
        self.ct.a_calls += 1
        return self.A @ X

    def chol(self, Om, k):
        R, ok = chol_flag(Om)
        if k in self.force_steps:
            ok = False
        return R, ok

    def start(self, R0, k=0):
        self.ct.syncs += muscle_syncs(self.muscle, self.s)
        Q, R, T, ok = intra_ortho(R0, self.muscle)
        if k in self.force_steps:
            ok = False
        return Q, R, T, ok

    def Hm1m(self, j: int) -> np.ndarray:
        """H_{j+1,j}-shaped leading block: rows of blocks 1..j+1, columns 1..j."""
        return self.H[: (j + 1) * self.s, : j * self.s]


class BMGS(_Skeleton):
    """BMGS-Arnoldi, Alg. 2 (Sec. 2.4): k inner products and subtractions per
    step, then IntraOrtho of the remainder."""

    def run(self, R0):
        V1, self.Beta, _, ok = self.start(R0)
        if not ok:
            self.flagged, self.last = True, 0
            return
        self.V = [V1]
        H = self.H
        for k in range(1, self.m + 1):
            W = self.matvec(self.V[k - 1])
            for i in range(1, k + 1):
                self.ct.syncs += 1
                H[self.blk(i), self.blk(k)] = self.ip(self.V[i - 1], W)
                W = W - self.V[i - 1] @ H[self.blk(i), self.blk(k)]
            self.ct.v_apps += 2
            self.ct.syncs += muscle_syncs(self.muscle, self.s)
            Q, R, _, ok = intra_ortho(W, self.muscle)
            if k in self.force_steps:
                ok = False
            if not ok:
                self.flagged, self.last = True, k - 1
                return
            H[self.blk(k + 1), self.blk(k)] = R
            self.V.append(Q)
            yield k


class BCGS_PIP(_Skeleton):
    """BCGS-PIP-Arnoldi, Alg. 3 (Sec. 3.1): one fused inner product
    [V_{1:k} W]^T W, Pythagorean Cholesky of Omega - H^T H, one projection."""

    def run(self, R0):
        V1, self.Beta, _, ok = self.start(R0)
        if not ok:
            self.flagged, self.last = True, 0
            return
        self.V = [V1]
        H, s = self.H, self.s
        for k in range(1, self.m + 1):
            W = self.matvec(self.V[k - 1])
            Vk = self.Vcat(k)
            self.ct.syncs += 1
            self.ct.v_apps += 2
            G = self.ip(np.hstack([Vk, W]), W)
            Hk = G[: k * s]
            Om = G[k * s:]
            H[self.upto(k), self.blk(k)] = Hk
            R, ok = self.chol(Om - Hk.T @ Hk, k)
            if not ok:
                self.flagged, self.last = True, k - 1
                return
            H[self.blk(k + 1), self.blk(k)] = R
            self.ct.v_apps += 1
            self.V.append(right_solve_upper(W - Vk @ Hk, R))
            yield k


class BCGS_PIO(_Skeleton):
    """BCGS-PIO-Arnoldi, Alg. 4 (Sec. 3.1): the block inner product
    H_{1:k,k} = V_{1:k}^T W, then the IntraOrtho of the block-diagonal
    matrix [W 0; 0 H_{1:k,k}] ((n + k s) x 2 s), whose R factor is block
    diagonal [R_W 0; 0 R_H]; H_{k+1,k} = chol(R_W^T R_W - R_H^T R_H) (the
    Pythagorean correction from the two triangular factors instead of the
    Gram blocks) and one projection.  Two syncs per step: the inner product
    and the IntraOrtho (Table 2: 2m + 1 per cycle).  A flag from the
    IntraOrtho or from the Cholesky stops the cycle with k - 1 final
    columns."""

    def run(self, R0):
        if self.muscle not in ("cholqr", "houseqr"):
            raise ValueError("BCGS-PIO is built here with the CholQR and HouseQR muscles only")
        V1, self.Beta, _, ok = self.start(R0)
        if not ok:
            self.flagged, self.last = True, 0
            return
        self.V = [V1]
        H, s = self.H, self.s
        for k in range(1, self.m + 1):
            W = self.matvec(self.V[k - 1])
            Vk = self.Vcat(k)
            self.ct.syncs += 1
            self.ct.v_apps += 1
            Hk = self.ip(Vk, W)
            H[self.upto(k), self.blk(k)] = Hk
            n = W.shape[0]
            D = np.zeros((n + k * s, 2 * s))
            D[:n, :s] = W
            D[n:, s:] = Hk
            self.ct.syncs += 1
            _, RD, _, ok = intra_ortho(D, self.muscle)
            if ok:
                RW, RH = RD[:s, :s], RD[s:, s:]
                R, ok = self.chol(RW.T @ RW - RH.T @ RH, k)
            elif k in self.force_steps:
                ok = False
            if not ok:
                self.flagged, self.last = True, k - 1
                return
            H[self.blk(k + 1), self.blk(k)] = R
            self.ct.v_apps += 1
            self.V.append(right_solve_upper(W - Vk @ Hk, R))
            yield k


class BMGS_SVL(_Skeleton):
    """BMGS-SVL / BMGS-LTS-Arnoldi, Alg. 5 (Sec. 3.2).

    SVL: H_{1:k,k} = T^T Y and T_{1:k,k+1} = -T Z T_{k+1,k+1};
    LTS: H_{1:k,k} = T^{-T} Y and T_{1:k,k+1} = Z T_{k+1,k+1}.

    Readings: T is allocated with (m+1) s rows/columns because step m writes
    T_{1:m,m+1}; T_{k+1,k+1} comes from the muscle (I_s for CholQR/HouseQR);
    Z is formed at every step including the last (the appendix's sync counts
    3 per iteration + 1 per cycle require it)."""

    lts = False

    def run(self, R0):
        m, s = self.m, self.s
        T = np.eye((m + 1) * s)
        V1, self.Beta, T11, ok = self.start(R0)
        if not ok:
            self.flagged, self.last = True, 0
            return
        T[self.blk(1), self.blk(1)] = T11
        self.V = [V1]
        H = self.H
        for k in range(1, m + 1):
            W = self.matvec(self.V[k - 1])
            Vk = self.Vcat(k)
            self.ct.syncs += 1
            self.ct.v_apps += 1
            Y = self.ip(Vk, W)
            Tk = T[self.upto(k), self.upto(k)]
            if self.lts:
                Hk = sla.solve_triangular(Tk.T, Y, lower=True, check_finite=False)
            else:
                Hk = Tk.T @ Y
            H[self.upto(k), self.blk(k)] = Hk
            self.ct.v_apps += 1
            Q, R, Tkk, ok = self.start(W - Vk @ Hk, k)
            if not ok:
                self.flagged, self.last = True, k - 1
                return
            H[self.blk(k + 1), self.blk(k)] = R
            T[self.blk(k + 1), self.blk(k + 1)] = Tkk
            self.V.append(Q)
            self.ct.syncs += 1
            self.ct.v_apps += 1
            Z = self.ip(Vk, Q)
            if self.lts:
                T[self.upto(k), self.blk(k + 1)] = Z @ Tkk
            else:
                T[self.upto(k), self.blk(k + 1)] = -(Tk @ Z) @ Tkk
            yield k


class BMGS_LTS(BMGS_SVL):
    lts = True


class BMGS_CWY(_Skeleton):
    """BMGS-CWY / BMGS-ICWY-Arnoldi, Alg. 6 (Sec. 3.3).

    CWY: T_{1:k-1,k} = -T_{1:k-1,1:k-1} (Y H_{k,k-1}^{-1}) and
         H_{1:k,k} = T_{1:k,1:k}^T ([Z;P] H_{k,k-1}^{-1});
    ICWY: T_{1:k-1,k} = Y H_{k,k-1}^{-1} and
          H_{1:k,k} = T_{1:k,1:k}^{-T} ([Z;P] H_{k,k-1}^{-1}).

    Readings: the two updates printed after the If-block (V_k = U H^{-1},
    U = W H^{-1} - V H) belong to the k >= 2 branch (at k = 1 there is no
    H_{1,0}, and the k = 1 branch already sets U); the product with
    H_{1:k,k} (k s rows) is taken with V_{1:k}, the basis including the
    just-formed V_k, as in Alg. 7."""

    delayed = True
    icwy = False

    def run(self, R0):
        m, s = self.m, self.s
        T = np.eye((m + 1) * s)
        V1, self.Beta, _, ok = self.start(R0)
        if not ok:
            self.flagged, self.last = True, 0
            return
        self.V = [V1]
        H = self.H
        U = V1
        for k in range(1, m + 2):
            W = self.matvec(U)
            if k == 1:
                self.ct.syncs += 1
                H[self.blk(1), self.blk(1)] = self.ip(U, W)
                self.ct.v_apps += 1
                U = W - self.V[0] @ H[self.blk(1), self.blk(1)]
                continue
            Vkm1 = self.Vcat(k - 1)
            self.ct.syncs += 1
            self.ct.v_apps += 2
            G = self.ip(np.hstack([Vkm1, U]), np.hstack([U, W]))
            Y, Z = G[: (k - 1) * s, :s], G[: (k - 1) * s, s:]
            Om, Pt = G[(k - 1) * s:, :s], G[(k - 1) * s:, s:]
            R, ok = self.chol(Om, k)
            if not ok:
                self.flagged, self.last = True, k - 2
                return
            H[self.blk(k), self.blk(k - 1)] = R
            P = left_solve_upper_t(R, Pt)
            YR = right_solve_upper(Y, R)
            if self.icwy:
                T[self.upto(k - 1), self.blk(k)] = YR
            else:
                T[self.upto(k - 1), self.blk(k)] = -(T[self.upto(k - 1), self.upto(k - 1)] @ YR)
            ZPR = right_solve_upper(np.vstack([Z, P]), R)
            Tk = T[self.upto(k), self.upto(k)]
            if self.icwy:
                H[self.upto(k), self.blk(k)] = sla.solve_triangular(Tk.T, ZPR, lower=True,
                                                                   check_finite=False)
            else:
                H[self.upto(k), self.blk(k)] = Tk.T @ ZPR
            self.V.append(right_solve_upper(U, R))
            self.ct.v_apps += 1
            U = right_solve_upper(W, R) - self.Vcat(k) @ H[self.upto(k), self.blk(k)]
            yield k - 1


class BMGS_ICWY(BMGS_CWY):
    icwy = True


class BCGSI_LS(_Skeleton):
    """BCGSI+LS-Arnoldi, Alg. 7 (Sec. 3.4): one fused inner product
    [V_{1:k-1} U]^T [U W] per step, with the Pythagorean correction
    Omega = Omega~ - Y^T Y, the auxiliary J, and delayed normalization.

    Reading: H_{1,1} = J set at k = 1 is provisional; the final
    H_{1:k-1,k-1} = J + Y is written at step k (before its Cholesky)."""

    delayed = True

    def run(self, R0):
        m, s = self.m, self.s
        V1, self.Beta, _, ok = self.start(R0)
        if not ok:
            self.flagged, self.last = True, 0
            return
        self.V = [V1]
        H = self.H
        U = V1
        J = None
        for k in range(1, m + 2):
            W = self.matvec(U)
            if k == 1:
                self.ct.syncs += 1
                J = self.ip(U, W)
                H[self.blk(1), self.blk(1)] = J
                self.ct.v_apps += 1
                U = W - self.V[0] @ J
                continue
            Vkm1 = self.Vcat(k - 1)
            self.ct.syncs += 1
            self.ct.v_apps += 2
            G = self.ip(np.hstack([Vkm1, U]), np.hstack([U, W]))
            Y, Z = G[: (k - 1) * s, :s], G[: (k - 1) * s, s:]
            Omt, Pt = G[(k - 1) * s:, :s], G[(k - 1) * s:, s:]
            Om = Omt - Y.T @ Y
            H[self.upto(k - 1), self.blk(k - 1)] = J + Y
            R, ok = self.chol(Om, k)
            if not ok:
                self.flagged, self.last = True, k - 2
                return
            H[self.blk(k), self.blk(k - 1)] = R
            P = left_solve_upper_t(R, Pt - Y.T @ Z)
            ZP = np.vstack([Z, P])
            J = right_solve_upper(ZP - H[self.upto(k), self.upto(k - 1)] @ Y, R)
            self.ct.v_apps += 1
            self.V.append(right_solve_upper(U - Vkm1 @ Y, R))
            self.ct.v_apps += 1
            U = right_solve_upper(W - self.Vcat(k) @ ZP, R)
            yield k - 1


SKELETONS = {
    "bmgs": BMGS,
    "bcgs_pip": BCGS_PIP,
    "bcgs_pio": BCGS_PIO,
    "bmgs_svl": BMGS_SVL,
    "bmgs_lts": BMGS_LTS,
    "bmgs_cwy": BMGS_CWY,
    "bmgs_icwy": BMGS_ICWY,
    "bcgsi_ls": BCGSI_LS,
}


def make_skeleton(name: str, A, s: int, m: int, muscle: str, counters: Counters | None = None,
                  force_steps=()):
    return SKELETONS[name](A, s, m, muscle, counters or Counters(), force_steps)
