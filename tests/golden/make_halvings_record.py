"""Writes cube12_halvings_PPN.json: for the FP64 oracle's PPN run over the
compressed heterogeneous cube at 12^3 cells (10,368 tets, 50 steps), every
Newton iteration of steps FIRST..50 with its accepted step size, the number of
elements it projected, whether its first solve met negative curvature, and the
three smallest eigenvalues of the matrix its final solve used (the assembled
Hessian at the iterate, with that iteration's projected elements replaced by
their projections, Eq. (5)).  It answers whether the steps that the line search
cuts (gamma < 1, Sec. 5.1) follow solves on matrices that are indefinite
although the PCG met no negative curvature.  Calls only the oracle and the
scene generator; dense eigenvalues (6,591 unknowns), about 20 minutes.
Run from the repository root:

    python tests/golden/make_halvings_record.py
"""
import json
import os
import sys

import numpy as np
import scipy.linalg

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle.fem import element_grad_hess  # noqa: E402
from oracle.project import project_to_pd  # noqa: E402
from scenes import cube_compress  # noqa: E402

N_CELLS = 12
FIRST = 35  # the halvings of this run fall on steps 42..50


def final_matrix(stp, x, projected_idx):
    """The matrix of an iteration's last solve: H(x) with the projected elements'
    Hessians replaced by their projections."""
    _, He = element_grad_hess(stp.mesh, x)
    H = stp.asm.hessian(He, stp._diag())
    sel = np.asarray(projected_idx, dtype=np.int64)
    if sel.size:
        Hhat = project_to_pd(He[sel], stp.p.eps_clamp, stp.p.eig_mirror)
        H = H + stp.asm.hessian(Hhat - He[sel], None, idx=sel)
    return H


def main():
    sc = cube_compress(n=N_CELLS, n_steps=50, ramp_steps=50)
    path = os.path.join(HERE, f"cube{N_CELLS}_halvings_PPN.json")
    out = {"scene": f"cube_compress(n={N_CELLS}, n_steps=50, ramp_steps=50)", "mode": "PPN",
           "steps_analysed": [FIRST, 50], "steps": []}

    def cb(n, stp, st):
        rec = dict(step=n, newton_iters=st.newton_iters, converged=bool(st.converged), iters=[])
        if n >= FIRST:
            for r in st.trace:
                if r.get("gamma") is None:  # the converged iterate: no solve
                    continue
                H = final_matrix(stp, r["x"], r["projected_idx"])
                lam = scipy.linalg.eigh(H.toarray(), eigvals_only=True, subset_by_index=[0, 2])
                rec["iters"].append(dict(k=r["k"], gamma=r["gamma"], n_projected=r["n_projected"],
                                         first_indefinite=bool(r["first"][0]), rounds=len(r["rounds"]),
                                         lambda_min=[float(v) for v in lam]))
        out["steps"].append(rec)
        with open(path + ".tmp", "w") as f:
            json.dump(out, f)
        os.replace(path + ".tmp", path)
        halved = [i for i in rec["iters"] if i["gamma"] < 1.0]
        print(n, st.newton_iters, "halvings", len(halved),
              [(i["k"], i["gamma"], i["n_projected"], round(i["lambda_min"][0], 4)) for i in halved], flush=True)

    oracle.run_scene(sc, "PPN", trace=True, record_x=True, callback=cb)


if __name__ == "__main__":
    main()
