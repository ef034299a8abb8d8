"""One backward-Euler time step by PN, PDN or PPN (oracle; test infrastructure only).

Newton's method (Sec. 3, Eq. (1)): solve H^k dx^k = -g^k, then x <- x + gamma dx.
* PN  projects every element Hessian before assembly (Sec. 3).
* PDN projects all element Hessians only once the assembled matrix is proven
  indefinite, then keeps projecting for a countdown of 4 iterations
  (Sec. 2.2 and Sec. 5.1).
* PPN (Algorithm 1) starts every iteration from the unprojected Hessian; on
  detected indefiniteness it projects the elements whose assembled local
  residual |S^e g|_inf exceeds delta, re-solves, tightens delta by alpha
  while the solve still detects indefiniteness, and relaxes it by beta once a
  descent direction is found.  delta starts at infinity, is initialised to
  alpha |g|_inf the first time projection is needed, and everything is
  projected once delta <= eps_delta (Sec. 4, projection heuristic).

Readings of points the paper leaves open:
* delta and the PDN countdown are reset at the start of each time step;
  within a step delta carries over Newton iterations.
* The Newton iterate starts at x^n; xhat = x^n + h v^n + h^2 g_grav; after the
  step v = (x - x^n)/h.
* Only elastic tetrahedra are candidates for projection; the inertia and
  penalty terms are SPD per vertex and never projected.
* S^e g takes the 12 entries of the assembled gradient at e's vertices;
  selection uses the strict comparison '>'.
* An element counts as projected when its Hessian is eigendecomposed, whether
  or not it had an eigenvalue below eps; already projected elements are not
  projected again within a Newton iteration.
* If the solve still reports indefiniteness with every element projected
  (possible only through rounding), the inner loop ends and the last PCG
  iterate is used if it is non-zero (a descent direction by the Newton-CG
  argument of Sec. 4.1), else -P^-1 g.
* Line search: Armijo backtracking, gamma = 1, 1/2, ..., at most 30 halvings,
  Psi(x + gamma dx) - Psi(x) <= c gamma g.dx with c = 1e-4; the energy
  difference is summed per term (per element and per vertex) to avoid
  cancellation.  If no trial passes, the step is not taken and the time step
  ends with an LS-failure flag.
* Stopping ("vel", Sec. 5.1): after the solve, stop when |dx|_inf / h < tol
  and do not apply that step.  "grad_rel": stop at the top of iteration k
  when |g^k|_2 <= tol |g^0|_2.  At most 100 Newton iterations.
* Dirichlet penalty stiffness k_D = 1e8 N/m; targets are those at the end of
  the step.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from .assemble import Assembler, diagonal_blocks
from .fem import Mesh, element_grad, element_grad_hess, element_psi, lumped_mass, predictor
from .pcg import pcg_block_jacobi
from .project import project_to_pd

MODES = ("PN", "PDN", "PPN")


@dataclass
class Params:
    alpha: float = 0.5          # tightening factor (Sec. 4)
    beta: float = 2.0           # release factor (Sec. 4)
    eps_delta: float = 1e-12    # PN fallback threshold (Sec. 4)
    eps_clamp: float = 1e-8     # eigenvalue clamp (Sec. 5.1)
    eig_mirror: bool = False    # mirror instead of clamp (Sec. 2, Sec. 5)
    pcg_rtol: float = 1e-4      # Sec. 5.1
    pcg_maxit: int = 10000
    pdn_countdown: int = 4      # Sec. 5.1
    stop_mode: str = "vel"
    stop_tol: float = 1e-3      # m/s (Sec. 5.1)
    newton_maxit: int = 100
    armijo_c: float = 1e-4
    ls_maxit: int = 30
    k_dirichlet: float = 1e8


@dataclass
class StepStats:
    newton_iters: int = 0
    pcg_iters: int = 0
    solves: int = 0
    indefinite_solves: int = 0
    inner_rounds: int = 0
    projected: int = 0
    ls_backtracks: int = 0
    safety_events: int = 0
    converged: bool = False
    ls_fail: bool = False
    res0_l2: float = 0.0
    res_l2: float = 0.0
    res_inf: float = 0.0
    trace: list = field(default_factory=list)


class Stepper:
    """Scene state plus the time-step solver."""

    def __init__(self, X, tets, E, nu, rho, dt, gravity, dirichlet_ids, params: Params,
                 x0=None, v0=None):
        self.mesh = Mesh.build(X, tets, E, nu)
        self.p = params
        self.h = float(dt)
        self.gravity = np.asarray(gravity, dtype=np.float64)
        self.m = lumped_mass(self.mesh, rho)
        self.asm = Assembler(self.mesh.tets, self.mesh.n_verts)
        self.dir_ids = np.asarray(dirichlet_ids, dtype=np.int64)
        self.xbar = np.asarray(X, dtype=np.float64)[self.dir_ids].copy()
        self.x = np.array(X if x0 is None else x0, dtype=np.float64)
        self.v = np.zeros_like(self.x) if v0 is None else np.array(v0, dtype=np.float64)
        self.xhat = None

    # ---- problem definition -------------------------------------------------
    def set_targets(self, xbar):
        self.xbar = np.asarray(xbar, dtype=np.float64).reshape(-1, 3).copy()

    def _vertex_gradient_terms(self, x):
        """Inertia m/h^2 (x - xhat) plus penalty k_D (x - xbar) per vertex."""
        t = (self.m / self.h ** 2)[:, None] * (x - self.xhat)
        t[self.dir_ids] += self.p.k_dirichlet * (x[self.dir_ids] - self.xbar)
        return t

    def _diag(self):
        d = np.repeat(self.m / self.h ** 2, 3)
        pen = np.zeros(self.mesh.n_verts)
        pen[self.dir_ids] = self.p.k_dirichlet
        return d + np.repeat(pen, 3)

    def evaluate(self, x):
        """(g (3N,), g^e, H^e, unprojected H) at x for the current step's xhat, xbar."""
        ge, He = element_grad_hess(self.mesh, x)
        g = self.asm.gradient(ge, self._vertex_gradient_terms(x))
        H = self.asm.hessian(He, self._diag())
        return g, ge, He, H

    def gradient(self, x):
        """Assembled g (3N,) at x without forming any Hessian."""
        return self.asm.gradient(element_grad(self.mesh, x), self._vertex_gradient_terms(x))

    def hessian_rows_product(self, x, d, rows, projected=None):
        """(H d) restricted to the vertex rows ``rows`` (k,3), from the elements
        incident to those rows only; elements in ``projected`` use Hhat^e."""
        rows = np.asarray(rows, dtype=np.int64)
        tets = self.mesh.tets
        inc = np.nonzero(np.isin(tets, rows).any(axis=1))[0]
        _, He = element_grad_hess(self.mesh, x, inc)
        if projected is not None:
            pm = np.zeros(self.mesh.n_tets, dtype=bool)
            pm[np.asarray(projected, dtype=np.int64)] = True
            sel = pm[inc]
            if sel.any():
                He[sel] = project_to_pd(He[sel], self.p.eps_clamp, self.p.eig_mirror)
        d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
        ye = np.einsum("tpq,tq->tp", He, d[tets[inc]].reshape(-1, 12)).reshape(-1, 4, 3)
        out = np.zeros((self.mesh.n_verts, 3))
        for a in range(4):
            np.add.at(out, tets[inc, a], ye[:, a])
        out += self._diag().reshape(-1, 3) * d
        return out[rows]

    def selection_residual(self, g):
        """|S^e g|_inf per element (Sec. 4, projection heuristic)."""
        gv = np.abs(g.reshape(-1, 3)).max(axis=1)
        return gv[self.mesh.tets].max(axis=1)

    def select(self, g, delta, projected):
        """Elements projected by one round of Algorithm 1's inner loop (Sec. 4):
        not projected yet in this Newton iteration, and |S^e g|_inf > delta
        (strict), or every such element once delta <= eps_delta."""
        return ~projected & ((self.selection_residual(g) > delta) | (delta <= self.p.eps_delta))

    def energy_difference(self, x, dx, gamma, psi_x=None):
        """Psi(x + gamma dx) - Psi(x), summed per term."""
        if psi_x is None:
            psi_x = element_psi(self.mesh, x)
        de = element_psi(self.mesh, x + gamma * dx) - psi_x
        step = gamma * dx
        di = (self.m / (2.0 * self.h ** 2)) * np.sum(step * (2.0 * (x - self.xhat) + step), axis=1)
        sd = step[self.dir_ids]
        dd = 0.5 * self.p.k_dirichlet * np.sum(sd * (2.0 * (x[self.dir_ids] - self.xbar) + sd), axis=1)
        return de.sum() + di.sum() + dd.sum()

    def line_search(self, x, dx, g):
        """Backtracking line search for sufficient descent (Sec. 5.1): try
        gamma = 1, 1/2, 1/4, ... and accept the first with
        Psi(x + gamma dx) - Psi(x) <= c gamma g.dx, after at most ls_maxit
        halvings.  Returns (gamma, accepted, rejected trials); after a failure
        every one of the ls_maxit + 1 trials was rejected."""
        p = self.p
        gdx = float(g @ dx.reshape(-1))
        psi_x = element_psi(self.mesh, x)
        gamma = 1.0
        for rejected in range(p.ls_maxit + 1):
            if self.energy_difference(x, dx, gamma, psi_x) <= p.armijo_c * gamma * gdx:
                return gamma, True, rejected
            gamma *= 0.5
        return gamma, False, p.ls_maxit + 1

    # ---- one time step ----------------------------------------------------------
    def step(self, mode: str, trace=False, record_x=False) -> StepStats:
        if mode not in MODES:
            raise ValueError(mode)
        p, h = self.p, self.h
        T = self.mesh.n_tets
        st = StepStats()
        x_n = self.x.copy()
        self.xhat = predictor(x_n, self.v, h, self.gravity)
        x = x_n.copy()
        delta = math.inf
        countdown = 0
        g0 = None

        for k in range(p.newton_maxit):
            st.newton_iters += 1
            g, _, He, H = self.evaluate(x)
            g_l2 = float(np.linalg.norm(g))
            g_inf = float(np.abs(g).max())
            st.res_l2, st.res_inf = g_l2, g_inf
            if k == 0:
                g0 = g_l2
                st.res0_l2 = g_l2
            rec = dict(k=k, g_l2=g_l2, g_inf=g_inf, delta_in=delta, rounds=[])
            if record_x:
                rec["x"] = x.copy()
            if p.stop_mode == "grad_rel" and g_l2 <= p.stop_tol * g0:
                st.converged = True
                if trace:
                    st.trace.append(rec)
                break

            projected = np.zeros(T, dtype=bool)
            state = {"H": H}

            def project(sel):
                sel = np.asarray(sel, dtype=np.int64)
                if sel.size == 0:
                    return
                Hhat = project_to_pd(He[sel], p.eps_clamp, p.eig_mirror)
                state["H"] = state["H"] + self.asm.hessian(Hhat - He[sel], None, idx=sel)
                projected[sel] = True
                st.projected += sel.size

            def solve():
                Hc = state["H"]
                dx, ind, it = pcg_block_jacobi(Hc, -g, diagonal_blocks(Hc), p.pcg_rtol, p.pcg_maxit)
                st.solves += 1
                st.pcg_iters += it
                st.indefinite_solves += int(ind)
                return dx, ind, it

            if mode == "PN" or (mode == "PDN" and countdown > 0):
                project(np.nonzero(~projected)[0])
                if mode == "PDN":
                    countdown -= 1
            rec["pre_projected"] = int(projected.sum())
            dx, ind, it = solve()
            rec["first"] = (bool(ind), it)
            if mode == "PDN" and ind and not projected.all():
                project(np.nonzero(~projected)[0])
                dx, ind, it = solve()
                countdown = p.pdn_countdown
            if mode == "PPN":
                while ind:
                    if delta == math.inf:
                        delta = p.alpha * g_inf
                    sel = np.nonzero(self.select(g, delta, projected))[0]
                    project(sel)
                    st.inner_rounds += 1
                    dx, ind, it = solve()
                    rec["rounds"].append((delta, int(sel.size), bool(ind), it))
                    if ind:
                        delta = p.alpha * delta
                    if ind and projected.all():
                        break
                delta = p.beta * delta
            if ind:
                st.safety_events += 1
                if not np.any(dx != 0.0):
                    blocks = diagonal_blocks(state["H"])
                    dx = -np.einsum("nij,nj->ni", np.linalg.inv(blocks), g.reshape(-1, 3)).reshape(-1)
            rec["n_projected"] = int(projected.sum())
            if trace:
                rec["projected_idx"] = np.nonzero(projected)[0].astype(np.int32)
            dxv = dx.reshape(-1, 3)
            dx_inf = float(np.abs(dxv).max())
            rec["dx_inf"] = dx_inf
            if p.stop_mode == "vel" and dx_inf / h < p.stop_tol:
                st.converged = True
                if trace:
                    st.trace.append(rec)
                break

            gamma, accepted, rejected = self.line_search(x, dxv, g)
            st.ls_backtracks += rejected
            rec["gamma"] = gamma if accepted else 0.0
            if trace:
                st.trace.append(rec)
            if not accepted:
                st.ls_fail = True
                break
            x = x + gamma * dxv

        self.v = (x - x_n) / h
        self.x = x
        return st


def run_scene(scene, mode, n_steps=None, params: Params = None, trace=False, callback=None, record_x=False):
    """Run ``n_steps`` time steps of a ``scenes.Scene``; returns (stepper, [StepStats]).
    With ``trace`` and ``record_x`` each iteration record also holds its iterate x^k."""
    if params is None:
        params = Params(stop_mode=scene.stop_mode, stop_tol=scene.stop_tol)
    stp = Stepper(scene.X, scene.tets, scene.E, scene.nu, scene.rho, scene.dt, scene.gravity,
                  scene.dirichlet_ids, params, x0=scene.x0, v0=scene.v0)
    out = []
    for n in range(1, (scene.n_steps if n_steps is None else n_steps) + 1):
        stp.set_targets(scene.targets(n))
        out.append(stp.step(mode, trace=trace, record_x=record_x))
        if callback is not None:
            callback(n, stp, out[-1])
    return stp, out
