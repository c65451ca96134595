"""Level data and the level operator A^l(x) (oracle; test infrastructure only).

A level holds, for each of its cells c (a fine cell on level 0, an aggregate
of the finer level otherwise):
  * its pressure coefficients (m_c of them; m_c = 1 on level 0),
  * its local flux degrees of freedom (global indices, ascending),
  * the static local matrix M_c (k_c x k_c) and the local divergence D_c
    (m_c x k_c),
  * the weights w_c of the piecewise-constant projector, so that the
    aggregate-average pressure of c is w_c . p_c (Appendix B, eq. pwc_projector;
    on level 0 the projector is the identity, so w_c = [1]).

With these, Section 3.2 (Prop. 1 and the remark after it) gives
    M^l(Pi~ p) = W^T  Mhat diag(W_sp kinv(Pi~ p))  W,
    A^l(x)     = [ M^l(Pi~ p) sigma + D^T p ;  D sigma ],
and Section 3.3 gives the Newton block
    E = N(sigma) diag(kinv'(Pi~ p)) Pi~ + D^T,  N(sigma) = W^T Mhat diag(W sigma) W_sp
(Props. 2 and 3).  W is the Boolean global-to-local flux map, W_sp the
local-flux-to-cell map; both are written out below exactly as defined.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

# flux degree-of-freedom kinds
INTERIOR, DIRICHLET, BUBBLE = 0, 1, 2


@dataclasses.dataclass
class Level:
    n_cells: int
    pdof_ptr: np.ndarray            # [n_cells+1]
    n_flux: int
    flux_kind: np.ndarray           # [n_flux] INTERIOR / DIRICHLET / BUBBLE
    flux_cells: np.ndarray          # [n_flux, 2]; second = -1 if only one cell
    cell_flux: List[np.ndarray]     # local flux dofs (global ids, ascending)
    M_loc: List[np.ndarray]         # static local matrices
    D_loc: List[np.ndarray]         # local divergence blocks
    w: List[np.ndarray]             # piecewise-constant projector weights
    ones: np.ndarray                # the vector 1^l (Appendix A.1)
    u: np.ndarray                   # volume moments u^l: (u^l)^T p = integral of the level-0 interpolant
    vol: np.ndarray                 # [n_cells] cell measures
    lattice_shape: Optional[tuple] = None
    lattice_index: Optional[np.ndarray] = None   # [n_cells]
    # shift z of the kappa argument per cell (kappa(Pi~ p - z)); level 0:
    # the problem's field, coarse levels: its volume-weighted mean over the
    # level-0 cells of each coarse cell.  None: no shift.
    shift: Optional[np.ndarray] = None
    # assembled operators (filled by finalize)
    W: Optional[sp.csr_matrix] = None
    Mhat: Optional[sp.csr_matrix] = None
    Wsp: Optional[sp.csr_matrix] = None
    D: Optional[sp.csr_matrix] = None
    Pi: Optional[sp.csr_matrix] = None

    @property
    def n_p(self) -> int:
        return int(self.pdof_ptr[-1])

    @property
    def n(self) -> int:
        return self.n_flux + self.n_p

    def pdofs(self, c: int) -> np.ndarray:
        return np.arange(self.pdof_ptr[c], self.pdof_ptr[c + 1])

    def finalize(self) -> "Level":
        """Build W, Mhat, W_sp, D and Pi~ from the per-cell data."""
        k = np.array([len(f) for f in self.cell_flux], dtype=np.int64)
        loc_ptr = np.concatenate([[0], np.cumsum(k)])
        nloc = int(loc_ptr[-1])
        rows = np.arange(nloc)
        cols = np.concatenate(self.cell_flux) if nloc else np.zeros(0, np.int64)
        self.W = sp.csr_matrix((np.ones(nloc), (rows, cols)), shape=(nloc, self.n_flux))
        self.Mhat = sp.block_diag(self.M_loc, format="csr") if nloc else sp.csr_matrix((0, 0))
        cell_of_loc = np.repeat(np.arange(self.n_cells), k)
        self.Wsp = sp.csr_matrix((np.ones(nloc), (rows, cell_of_loc)), shape=(nloc, self.n_cells))
        dr, dc, dv = [], [], []
        pr, pc, pv = [], [], []
        for c in range(self.n_cells):
            pd = self.pdofs(c)
            Dc = self.D_loc[c]
            rr, cc = np.meshgrid(pd, self.cell_flux[c], indexing="ij")
            dr.append(rr.ravel()); dc.append(cc.ravel()); dv.append(Dc.ravel())
            pr.append(np.full(pd.size, c)); pc.append(pd); pv.append(self.w[c])
        self.D = sp.csr_matrix((np.concatenate(dv), (np.concatenate(dr), np.concatenate(dc))),
                               shape=(self.n_p, self.n_flux))
        self.Pi = sp.csr_matrix((np.concatenate(pv), (np.concatenate(pr), np.concatenate(pc))),
                                shape=(self.n_cells, self.n_p))
        return self


# ------------------------------------------------------------- kappa family

@dataclasses.dataclass(frozen=True)
class Kappa:
    """The scalar multiplier kappa of K(x, p) = K0(x) kappa (eq. kappa), as a
    function of the shifted pressure psi = p - z(x):
      * "exp":      kappa(psi) = exp(alpha psi) (Section 2, the model problem);
      * "richards": kappa(psi) = a / (a + |psi|^beta) (Example 3, eq.
        permeability_function_richards, with the pressure head psi = p - z
        and z the height; the paper's alpha is ``a`` here).
    The shift z is a per-cell field of the level (``Level.shift``); None is
    z = 0.  Only 1/kappa and its derivative enter the method (Prop. 1,
    Props. 2-3)."""
    kind: str = "exp"
    alpha: float = 0.0
    a: float = 1.0
    beta: float = 2.0

    def kinv(self, psi: np.ndarray) -> np.ndarray:
        if self.kind == "exp":
            return np.exp(-self.alpha * psi)
        if self.kind == "richards":
            return 1.0 + np.abs(psi) ** self.beta / self.a
        raise ValueError(f"unknown kappa family {self.kind!r}")

    def dkinv(self, psi: np.ndarray) -> np.ndarray:
        """d(1/kappa)/d psi."""
        if self.kind == "exp":
            return -self.alpha * np.exp(-self.alpha * psi)
        if self.kind == "richards":
            return np.sign(psi) * self.beta * np.abs(psi) ** (self.beta - 1.0) / self.a
        raise ValueError(f"unknown kappa family {self.kind!r}")


def as_kappa(alpha) -> Kappa:
    """A number is the exponent of the exponential family."""
    return alpha if isinstance(alpha, Kappa) else Kappa("exp", float(alpha))


def kappa_of(prob):
    """The kappa model of a problem: its alpha for the plain exponential,
    else a Kappa."""
    kind = getattr(prob, "kappa_kind", "exp")
    if kind == "exp":
        return prob.alpha
    return Kappa(kind, prob.alpha, getattr(prob, "kappa_a", 1.0), getattr(prob, "kappa_beta", 2.0))


def kinv(pbar: np.ndarray, alpha) -> np.ndarray:
    """1/kappa(p) for kappa(p) = exp(alpha p) (Section 2, eq. for kappa), or
    for the family of a Kappa."""
    if isinstance(alpha, Kappa):
        return alpha.kinv(pbar)
    return np.exp(-alpha * pbar)


def dkinv(pbar: np.ndarray, alpha) -> np.ndarray:
    """d(1/kappa)/dp for kappa(p) = exp(alpha p), or for a Kappa."""
    if isinstance(alpha, Kappa):
        return alpha.dkinv(pbar)
    return -alpha * np.exp(-alpha * pbar)


# ------------------------------------------------------------- operators

def split(level: Level, x: np.ndarray):
    return x[:level.n_flux], x[level.n_flux:]


def pwc(level: Level, p: np.ndarray) -> np.ndarray:
    """Aggregate-average pressure Pi~ p, one value per cell (Appendix B)."""
    return level.Pi @ p


def psi_of(level: Level, p: np.ndarray) -> np.ndarray:
    """The argument of kappa per cell: Pi~ p minus the level's shift."""
    pb = pwc(level, p)
    return pb if level.shift is None else pb - level.shift


def M_of(level: Level, p: np.ndarray, alpha: float) -> sp.csr_matrix:
    """M^l(Pi~ p) = W^T Mhat diag(W_sp kinv(Pi~ p)) W (Prop. 1, eq. assemble)."""
    s = level.Wsp @ kinv(psi_of(level, p), alpha)
    return (level.W.T @ (level.Mhat @ sp.diags(s)) @ level.W).tocsr()


def apply_A(level: Level, x: np.ndarray, alpha: float) -> np.ndarray:
    """A^l(x) = [M(Pi~ p) sigma + D^T p; D sigma] (eq. structure)."""
    sig, p = split(level, x)
    return np.concatenate([M_of(level, p, alpha) @ sig + level.D.T @ p, level.D @ sig])


def residual(level: Level, x: np.ndarray, b: np.ndarray, alpha: float) -> np.ndarray:
    """r^l(x) = A^l(x) - b^l (eq. nonlinear_system_level_l)."""
    return apply_A(level, x, alpha) - b


def N_of(level: Level, sig: np.ndarray) -> sp.csr_matrix:
    """N(sigma) = W^T Mhat diag(W sigma) W_sp (Prop. 2, eq. definition-N)."""
    return (level.W.T @ level.Mhat @ sp.diags(level.W @ sig) @ level.Wsp).tocsr()


def E_of(level: Level, x: np.ndarray, alpha: float, newton: bool) -> sp.csr_matrix:
    """E = D^T (Picard) or d r_sigma / dp = N(sigma) kinv'(Pi~p) Pi~ + D^T
    (Newton, Prop. 3, eq. d_flux_residual_d_pk)."""
    sig, p = split(level, x)
    E = level.D.T.tocsr()
    if newton:
        E = E + N_of(level, sig) @ sp.diags(dkinv(psi_of(level, p), alpha)) @ level.Pi
    return E.tocsr()


def jacobian(level: Level, x: np.ndarray, alpha: float, newton: bool) -> sp.csr_matrix:
    """[M E; D 0] (eq. general-block-system): Picard with E = D^T (eq.
    picardian_system), Newton with the full derivative (eq. jacobian_matrix)."""
    sig, p = split(level, x)
    M = M_of(level, p, alpha)
    E = E_of(level, x, alpha, newton)
    Z = sp.csr_matrix((level.n_p, level.n_p))
    return sp.bmat([[M, E], [level.D, Z]], format="csc")
