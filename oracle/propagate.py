"""CPU oracle of a fixed-grid two-time propagation of the Kadanoff-Baym equations and of its
gradients (TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's CPU
baseline use it; the GPU library shares no code with it).

Plain PyTorch on the CPU in complex128.  Every sum is written as its definition with einsum /
matmul as the only library steps; the gradient of a loss is torch.autograd through this forward
code, so the "oracle adjoint" is an independent derivation of the same discrete map.  The
quadrature weights come from the pinned C oracle (oracle.weights, oracle.local_weights,
oracle.tau_weights): they depend on the grid only and are not differentiated.

The discrete map (arXiv:2405.08737, Sec. "Kadanoff Baym Equations" and Sec. "Adaptive Time
Stepping", specialised to a fixed grid and fixed orders):

Unknowns, in the KP storage of the GPU library: kp[m][n] = G^<(t_m,t_n) (m <= n), kp[n][m] =
G^R(t_n,t_m) (m < n), rdiag = G^R(t,t) = -i (Eq. BC), tv[n][j] = G^](t_n,tau_j); G^M = mat is
the initial condition.  The paper propagates G^< above the diagonal and G^> below it, stacked as
one state vector in a single time variable t~ (the new row and column at t_n = t~).  With
G^R = G^> - G^< below the diagonal this is, per element, the ODE in t~ of
  U_m : G^<(t_m, t~)   f = d/dt' G^<(t_m,t')  = i (G^<(t_m,t~) eps(t~) - C^<(t~,t_m)^dagger)   (Eq. KBE1)
  R_m : G^R(t~, t_m)   f = d/dt G^>(t,t_m) - d/dt G^<(t,t_m)
                         = -i (eps(t~) G^R(t~,t_m) + C^>(t~,t_m) - C^<(t~,t_m))             (Eq. KBE2)
  D   : G^<(t~, t~)    f = -i [eps, G^<(t~,t~)] - i (C^<(t~,t~) + C^<(t~,t~)^dagger)
  T_j : G^](t~, tau_j) f = -i (eps(t~) G^](t~,tau_j) + J^](t~,tau_j))                        (Eq. KBE3)
where C^< = I^R + I^< + I^] is the history sum of the lesser form of Eq. KBE2 at (t_n, t_m)
(KBE1's integrals at (t_m,t_n) are its negative adjoint), C^> the same sum of the greater form
(G^> in I^R, Sigma^> in I^<), J^] the history terms of Eq. KBE3, Sigma the local-U second-Born
self-energy of Eq. SE, and eps the Fock matrix of Eq. eps with a local U,
  eps(t) = h0 + p(t) e_00 + diag(-i u_i G^<_ii(t,t)),   p(t) = A exp(-(t - t_c)^2 / (2 sigma^2)),
the Gaussian pulse on h_00.  U_m and R_m are born at t~ = t_m with G^<(t_m,t_m) and -i.

Time stepping: each element advances over interval n = [t_{n-1}, t_n] by the implicit
Adams-Moulton rule in Lagrange form, y_n = y_{n-1} + sum_i lam_i f(t_{n-k+1+i}), with the local
weights lam of Eq. weights for interval n on the nodes t_{n-k+1..n} (the history integrals'
weights) and k = min(order[n], n - b + 1) nodes for an element born at t_b (the rule uses only the
element's own history).  The implicit equation is solved by a fixed number K of fixed-point
iterations from the explicit Euler predictor y^(0) = y_{n-1} + (t_n - t_{n-1}) f(t_{n-1}):
y^(i) = y_{n-1} + sum_{i<k-1} lam_i f_i + lam_{k-1} f(y^(i-1)); the f values stored for later
steps are evaluated once more at y^(K) (the paper also re-evaluates Sigma at the accepted
solution).  Observable: the densities n_i(t_n) = Re(-i G^<_ii(t_n,t_n)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

import oracle as _orc

CT = torch.complex128


def H(x):
    """Conjugate transpose of the last two axes."""
    return x.conj().transpose(-1, -2)


@dataclass
class Problem:
    t: np.ndarray            # [nt] grid, t[0] = 0
    order: np.ndarray        # [nt] nodes per interval (history weights and time stepping)
    h0: np.ndarray           # [N][N] real symmetric
    ntau: int                # imaginary-time points (0: no thermal branch)
    beta: float = 1.0
    tau_order: int = 5
    mat: np.ndarray | None = None   # [ntau][N][N] G^M (initial condition, ntau > 0)
    rho0: np.ndarray | None = None  # [N][N] initial density matrix (ntau == 0)
    iters: int = 2           # fixed-point iterations per step
    pulse_t0: float = 2.0
    pulse_sigma: float = 1.0
    _w: dict = field(default_factory=dict, repr=False)

    @property
    def N(self):
        return self.h0.shape[0]

    @property
    def nt(self):
        return len(self.t)

    def weights(self):
        if "w" not in self._w:
            self._w["w"] = torch.tensor(_orc.weights(self.t, self.order))
            if self.ntau:
                wf, wb, wfull = _orc.tau_weights(self.beta, self.ntau, self.tau_order)
                self._w["tau"] = tuple(torch.tensor(x) for x in (wf, wb, wfull))
            lam = {}
            for n in range(1, self.nt):
                for k in range(1, min(int(self.order[n]), n + 1) + 1):
                    lam[(n, k)] = torch.tensor(_orc.local_weights(self.t, n, k))
            self._w["lam"] = lam
        return self._w


def initial_state(P: Problem):
    """G^<(0,0) and G^](0,tau_j) from Eq. BC: G^](0,tau) = i G^M(-tau) = -i G^M(beta - tau) and
    G^<(0,0) = -G^](0,0)^dagger; without a thermal branch G^<(0,0) = i rho0."""
    N = P.N
    if P.ntau:
        mat = torch.tensor(P.mat, dtype=CT)
        J = P.ntau - 1
        tv0 = torch.stack([-1j * mat[J - j] for j in range(P.ntau)])
        d0 = -H(tv0[0])
    else:
        tv0 = torch.zeros((0, N, N), dtype=CT)
        d0 = 1j * torch.tensor(P.rho0, dtype=CT)
    return d0, tv0


# ---------------------------------------------------------------------------------------------
# Self-energy row and history sums on a dense copy of the KP storage (rows/cols 0..n).
# ---------------------------------------------------------------------------------------------
def views(KP, N):
    """(GL, GR, GG) for indices 0..n from KP [n+1][n+1][N][N]: GL[s][m] = G^<(t_s,t_m),
    GR[a][b] = G^R(t_a,t_b) for a > b, -i on the diagonal and 0 above, GG[s][m] = G^>(t_s,t_m)."""
    n1 = KP.shape[0]
    idx = torch.arange(n1)
    up = (idx[:, None] <= idx[None, :])[:, :, None, None]
    low = (idx[:, None] > idx[None, :])[:, :, None, None]
    dg = (idx[:, None] == idx[None, :])[:, :, None, None]
    eye = torch.eye(N, dtype=CT)
    KPT = KP.transpose(0, 1)
    GL = torch.where(up, KP, -H(KPT))
    GR = torch.where(low, KP, torch.zeros_like(KP)) + dg * (-1j * eye)
    GGlow = GR + GL                          # G^> = G^R + G^< for s >= m
    GG = torch.where(up & ~dg, -H(GGlow.transpose(0, 1)), GGlow)
    return GL, GR, GG


def sigma_row(GL, GG, tvn, u, n):
    """Local-U second Born (Eq. SE with U_ijkl = u_i d_ij d_jk d_kl):
    Sigma^<>_ij(t,t') = u_i u_j G^<>_ij(t,t')^2 G^><_ji(t',t), Sigma^]_ij(t,tau) = u_i u_j
    G^]_ij(t,tau)^2 conj(G^]_ij(t,beta-tau)).  Returns (ret = Sigma^> - Sigma^<, les, stv) at t_n."""
    uu = (u[:, None] * u[None, :]).to(CT)
    Sl = uu * GL[n] ** 2 * GG[:, n].transpose(-1, -2)
    Sg = uu * GG[n] ** 2 * GL[:, n].transpose(-1, -2)
    stv = uu * tvn ** 2 * tvn.flip(0).conj()
    return Sg - Sl, Sl, stv


def collision(GL, GR, GG, TV, mat, sig, W, n, greater=False):
    """History sums of row n for m = 0..n (Eq. KBE2; lesser form, or greater form), and J^]
    (Eq. KBE3).  Returns (IR, IL, Itv, Jtv)."""
    ret, les, stv = sig
    w = W["w"]
    wn = w[n, : n + 1].to(CT)
    wm = w[: n + 1, : n + 1].to(CT)          # w[m][s] = 0 for s > m
    G = GG if greater else GL
    Q = ret + les if greater else les
    IR = torch.einsum("s,sij,smjk->mik", wn, ret, G)
    IL = torch.einsum("ms,sij,mskj->mik", wm, Q, GR.conj())
    if TV.shape[1] == 0:
        z = torch.zeros((0, *ret.shape[1:]), dtype=CT)
        return IR, IL, torch.zeros_like(IR), z
    wf, wb, wfull = W["tau"]
    ntau = TV.shape[1]
    J = ntau - 1
    Itv = -1j * torch.einsum("j,jab,mjcb->mac", wfull.to(CT), stv, TV.flip(1).conj())
    Jtv = torch.einsum("s,sab,sjbc->jac", wn, ret, TV)
    jj = torch.arange(ntau)
    for j in range(ntau):   # Matsubara convolution split at tau_j
        cl = torch.where(jj <= j, -wf[j], torch.zeros_like(wf[j])).to(CT)
        cg = torch.where(jj >= j, wb[j], torch.zeros_like(wb[j])).to(CT)
        Mlo = mat[(J + jj - j).clamp(0, J)]
        Mhi = mat[(jj - j).clamp(0, J)]
        Jtv = Jtv + torch.cat([torch.zeros((j, *ret.shape[1:]), dtype=CT),
                               (torch.einsum("l,lab,lbc->ac", cl, stv, Mlo)
                                + torch.einsum("l,lab,lbc->ac", cg, stv, Mhi))[None],
                               torch.zeros((ntau - j - 1, *ret.shape[1:]), dtype=CT)])
    return IR, IL, Itv, Jtv


# ---------------------------------------------------------------------------------------------
# The propagation.
# ---------------------------------------------------------------------------------------------
class State:
    """The stored solution as lists of tensors (so autograd sees every value once):
    col[n] [n+1]: kp[m][n], m <= n;  row[n] [n]: kp[n][m], m < n;  tv[n] [ntau]."""

    def __init__(self, N, ntau):
        self.N, self.ntau = N, ntau
        self.col, self.row, self.tv = [], [], []

    def dense(self, n, col_n, row_n, tv_n):
        """KP [n+1][n+1] and TV [n+1][ntau] with row/column n taken from the given tensors."""
        N = self.N
        cols = [torch.cat([c, torch.zeros((n - len(c) + 1, N, N), dtype=CT)])
                for c in self.col[:n]] + [col_n]
        rows = [torch.cat([r, torch.zeros((n - len(r) + 1, N, N), dtype=CT)])
                for r in self.row[:n]] + [torch.cat([row_n, torch.zeros((1, N, N), dtype=CT)])]
        Up = torch.stack(cols).transpose(0, 1)        # Up[a][b] = col[b][a]
        Lo = torch.stack(rows)                        # Lo[a][b] = row[a][b]
        idx = torch.arange(n + 1)
        KP = torch.where((idx[:, None] <= idx[None, :])[:, :, None, None], Up, Lo)
        TV = torch.stack(self.tv[:n] + [tv_n]) if self.ntau else \
            torch.zeros((n + 1, 0, N, N), dtype=CT)
        return KP, TV


def rhs(P: Problem, S: State, n, col_n, row_n, tv_n, u, A, mat, W=None, tn=None, choose=None):
    """f of every element of step n at the given row/column n: (fU [n] for m < n, fR [n],
    fD, fT [ntau], fbu, fbr) with fbu / fbr the derivatives at birth of U_n and R_n.
    W (default P.weights()) holds the history weights; tn (default P.t[n]) the time; choose, when
    given, is called with (GL, GR, Sigma row) before the history sums and may set W's row n (the
    adaptive history order)."""
    N = P.N
    W = P.weights() if W is None else W
    KP, TV = S.dense(n, col_n, row_n, tv_n)
    GL, GR, GG = views(KP, N)
    D = col_n[n]
    tn = float(P.t[n]) if tn is None else float(tn)
    pulse = torch.exp(torch.tensor(-(tn - P.pulse_t0) ** 2 / (2 * P.pulse_sigma ** 2),
                                   dtype=torch.float64))
    e00 = torch.zeros((N, N), dtype=CT)
    e00[0, 0] = 1.0
    eps = torch.tensor(P.h0, dtype=CT) + (A * pulse).to(CT) * e00 + \
        torch.diag(-1j * u.to(CT) * torch.diagonal(D))
    sig = sigma_row(GL, GG, tv_n, u, n)
    if choose is not None:
        choose(GL, GR, sig)
    IRl, ILl, Itv, Jtv = collision(GL, GR, GG, TV, mat, sig, W, n, greater=False)
    IRg, ILg, _, _ = collision(GL, GR, GG, TV, mat, sig, W, n, greater=True)
    Cl = IRl + ILl + Itv
    Cg = IRg + ILg + Itv
    Ucol = col_n[:n]                                      # G^<(t_m,t_n), m < n
    fU = 1j * (Ucol @ eps - H(Cl[:n]))
    fR = -1j * (eps @ row_n + Cg[:n] - Cl[:n])
    fD = -1j * (eps @ D - D @ eps) - 1j * (Cl[n] + H(Cl[n]))
    fT = -1j * (eps @ tv_n + Jtv) if P.ntau else tv_n
    fbu = 1j * (D @ eps - H(Cl[n]))
    fbr = -1j * (eps @ (-1j * torch.eye(N, dtype=CT)) + Cg[n] - Cl[n])
    return fU, fR, fD, fT, fbu, fbr


def propagate(P: Problem, U, A, *, keep=False):
    """Run the propagation.  U: scalar tensor (uniform local interaction, u_i = U) or [N] tensor;
    A: scalar tensor (pulse amplitude).  Returns (dens [nt][N] tensor, State)."""
    N, nt, K = P.N, P.nt, P.iters
    W = P.weights()
    lam = W["lam"]
    u = U * torch.ones(N, dtype=torch.float64) if U.dim() == 0 else U
    mat = torch.tensor(P.mat, dtype=CT) if P.ntau else torch.zeros((0, N, N), dtype=CT)
    S = State(N, P.ntau)
    d0, tv0 = initial_state(P)
    # f histories: fU[m] list over t_j >= t_m (index 0 = birth), fR[m] likewise, fD, fT lists
    fU, fR, fD, fT = [], [], [], []
    col0, row0 = d0[None], torch.zeros((0, N, N), dtype=CT)
    f = rhs(P, S, 0, col0, row0, tv0, u, A, mat)
    S.col.append(col0)
    S.row.append(row0)
    S.tv.append(tv0)
    fU.append([f[4]])
    fR.append([f[5]])
    fD.append(f[2])
    fT.append(f[3])
    dens = [torch.real(-1j * torch.diagonal(d0))]
    for n in range(1, nt):
        kn = int(P.order[n])
        h = float(P.t[n] - P.t[n - 1])
        # element values at t_{n-1} and their Adams-Moulton bases and predictors
        prevU = S.col[n - 1]                              # [n]: U_m for m <= n-1 (m = n-1: D)
        prevR = torch.cat([S.row[n - 1], (-1j * torch.eye(N, dtype=CT))[None]])  # R_m, m <= n-1
        prevD = S.col[n - 1][n - 1]
        prevT = S.tv[n - 1]

        def am(prev, hist, b):
            """(base, lam_last, predictor) for an element born at t_b with f history hist
            (hist[j - b] = f at t_j, j = b..n-1)."""
            k = min(kn, n - b + 1)
            lk = lam[(n, k)]
            base = prev
            for i in range(k - 1):
                base = base + lk[i].item() * hist[n - k + 1 + i - b]
            return base, lk[k - 1].item(), prev + h * hist[n - 1 - b]

        bU, lU, pU = zip(*[am(prevU[m], fU[m], m) for m in range(n)])
        bR, lR, pR = zip(*[am(prevR[m], fR[m], m) for m in range(n)])
        bD, lD, pD = am(prevD, fD, 0)
        if P.ntau:
            bT, lT, pT = am(prevT, fT, 0)
        bU, bR, pU, pR = (torch.stack(x) for x in (bU, bR, pU, pR))
        lU = torch.tensor(lU, dtype=CT)[:, None, None]
        lR = torch.tensor(lR, dtype=CT)[:, None, None]
        yU, yR, yD = pU, pR, pD
        yT = pT if P.ntau else prevT
        for _ in range(K):
            col_n = torch.cat([yU, yD[None]])
            f = rhs(P, S, n, col_n, yR, yT, u, A, mat)
            yU = bU + lU * f[0]
            yR = bR + lR * f[1]
            yD = bD + lD * f[2]
            if P.ntau:
                yT = bT + lT * f[3]
        col_n = torch.cat([yU, yD[None]])
        f = rhs(P, S, n, col_n, yR, yT, u, A, mat)
        S.col.append(col_n)
        S.row.append(yR)
        S.tv.append(yT)
        for m in range(n):
            fU[m].append(f[0][m])
            fR[m].append(f[1][m])
        fU.append([f[4]])
        fR.append([f[5]])
        fD.append(f[2])
        fT.append(f[3])
        dens.append(torch.real(-1j * torch.diagonal(yD)))
    return torch.stack(dens), S


def storage(S: State):
    """The solution as numpy KP storage (kp [nt][nt][N][N], tv [nt][ntau][N][N])."""
    nt = len(S.col)
    N = S.N
    kp = np.zeros((nt, nt, N, N), np.complex128)
    for n in range(nt):
        c = S.col[n].detach().numpy()
        r = S.row[n].detach().numpy()
        kp[: n + 1, n] = c
        kp[n, :n] = r
    tv = np.stack([x.detach().numpy() for x in S.tv]) if S.ntau else \
        np.zeros((nt, 0, N, N), np.complex128)
    return kp, tv


def loss_and_grad(P: Problem, U: float, A: float, c, last: int):
    """L = sum over the last `last` steps and orbitals of c_i n_i(t_n), and (dL/dU, dL/dA) by
    reverse-mode differentiation of propagate()."""
    Ut = torch.tensor(U, dtype=torch.float64, requires_grad=True)
    At = torch.tensor(A, dtype=torch.float64, requires_grad=True)
    dens, _ = propagate(P, Ut, At)
    L = (dens[-last:] * torch.tensor(np.asarray(c, np.float64))).sum()
    gU, gA = torch.autograd.grad(L, [Ut, At])
    return L.item(), gU.item(), gA.item()


def loss(P: Problem, U: float, A: float, c, last: int) -> float:
    with torch.no_grad():
        dens, _ = propagate(P, torch.tensor(U, dtype=torch.float64),
                            torch.tensor(A, dtype=torch.float64))
    return float((dens[-last:] * torch.tensor(np.asarray(c, np.float64))).sum())
