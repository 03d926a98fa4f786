"""Near-critical hopping parameter of a synthetic configuration (oracle).

TEST / WORKLOAD INFRASTRUCTURE.  M = 1 - kappa P is affine in kappa, so its
eigenvalues are lambda = 1 - kappa mu with mu the eigenvalues of P
(Sec. 5.1 Eq. (24)); the smallest real part of the spectrum of M equals
delta when kappa = (1 - delta) / max Re mu(P).  The rightmost eigenvalue of
P is found with ARPACK (implicitly restarted Arnoldi, which = 'LR') on the
oracle's stencil (its plain-C form, oracle/c/hop.c, for speed), from a
seeded start vector; the returned eigenpair is then checked with the numpy
stencil (relative residual |P v - mu v| / |mu| reported).

Run:  python -m oracle.critical_kappa c3      (writes synth/c3_kappa.json)
"""
import json
import os
import sys
import time

import numpy as np


def rightmost_eig(U, dims, tol=1e-7, ncv=24, seed=0, fast=True, progress=0):
    """Two rightmost eigenvalues of P, the eigenvector of the first, and the
    number of products with P."""
    import scipy.sparse.linalg as sla
    from .wilson import hop
    from .chop import hop_c
    Lx, Ly, Lz, Lt = dims
    shape = (Lt, Lz, Ly, Lx, 4, 3)
    n = 12 * Lx * Ly * Lz * Lt
    count = [0]
    t0 = time.time()
    f = hop_c if fast else hop

    def mv(v):
        count[0] += 1
        if progress and count[0] % progress == 0:
            print("[kappa] %d products with P, %.0f s" % (count[0], time.time() - t0), flush=True)
        return f(U, v.reshape(shape)).ravel()

    op = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    vals, vecs = sla.eigs(op, k=2, which="LR", ncv=ncv, tol=tol, v0=v0)
    order = np.argsort(-vals.real)
    return vals[order], vecs[:, order[0]], count[0]


def main(name):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import get_config, random_su3_links
    cfg = get_config(name)
    dims = cfg["dims"]
    U = random_su3_links(dims, cfg["eps"], cfg["link_seed"])
    from .wilson import hop
    t0 = time.time()
    tol, ncv = 1e-6, 48
    vals, vec, nmv = rightmost_eig(U, dims, tol=tol, ncv=ncv, progress=500)
    shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
    v = vec.reshape(shape)
    resid = float(np.linalg.norm(hop(U, v) - vals[0] * v) / (abs(vals[0]) * np.linalg.norm(v)))
    mu = float(vals[0].real)
    delta = cfg.get("delta", 1e-3)
    out = dict(config=name, dims=list(dims), eps=cfg["eps"], link_seed=cfg["link_seed"],
               rightmost_mu=[[float(v.real), float(v.imag)] for v in vals],
               max_re_mu=mu, eig_resid=resid, delta=delta, kappa=(1.0 - delta) / mu, matvecs=nmv,
               seconds=time.time() - t0,
               method="ARPACK eigs(which='LR', k=2, ncv=%d, tol=%g) on the oracle hop" % (ncv, tol))
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "synth",
                        "%s_kappa.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c3")
