"""Near-critical hopping parameter of a synthetic configuration (oracle).

TEST / WORKLOAD INFRASTRUCTURE.  M = 1 - kappa P is affine in kappa, so its
eigenvalues are lambda = 1 - kappa mu with mu the eigenvalues of P
(Sec. 5.1 Eq. (24)); the smallest real part of the spectrum of M equals
delta when kappa = (1 - delta) / max Re mu(P).  The rightmost eigenvalue of
P is found with ARPACK (implicitly restarted Arnoldi, which = 'LR') on the
oracle's stencil (its plain-C form, oracle/c/hop.c, for speed), from a
seeded start vector; the returned eigenpair is then checked with the numpy
stencil (relative residual |P v - mu v| / |mu| reported).

On large lattices the search runs on the even/odd square D_eo D_oe (even
sites) instead: P maps even to odd sites and back, so P^2 is block
diagonal and its even block has the eigenvalues mu^2 (each pair +-mu of P
maps to one mu^2).  For a real rightmost mu, mu^2 is the rightmost
eigenvalue of the block (Re mu^2 = a^2 - b^2 is largest on the real
edge), the vectors are half as long and the edge is relatively better
separated.  The eigenvector v_e of mu^2 gives the eigenvector
v = (v_e, D_oe v_e / mu) of P, whose residual is checked with the numpy
stencil, so a complex or misidentified edge fails that check.

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


def rightmost_eig_eo(U, dims, tol=1e-7, ncv=24, seed=0, progress=0, k=2):
    """Rightmost eigenvalue of P through its even/odd square: returns (mu,
    eigenvalues of D_eo D_oe found, eigenvector of P, products with P)."""
    import scipy.sparse.linalg as sla
    from .chop import hop_c
    from .lattice import parity as lat_parity
    Lx, Ly, Lz, Lt = dims
    shape = (Lt, Lz, Ly, Lx, 4, 3)
    even = np.broadcast_to((lat_parity(dims) == 0)[..., None, None], shape)
    ne = int(even.sum())
    count = [0]
    t0 = time.time()

    def mv(v):
        count[0] += 2
        if progress and count[0] % progress == 0:
            print("[kappa] %d products with P (even/odd square), %.0f s" % (count[0], time.time() - t0),
                  flush=True)
        full = np.zeros(shape, dtype=np.complex128)
        full[even] = v
        odd = hop_c(U, full, parity=1)       # D_oe v_e
        return hop_c(U, odd, parity=0)[even]  # D_eo D_oe v_e

    op = sla.LinearOperator((ne, ne), matvec=mv, dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(ne) + 1j * rng.standard_normal(ne)
    vals, vecs = sla.eigs(op, k=k, which="LR", ncv=ncv, tol=tol, v0=v0)
    order = np.argsort(-vals.real)
    nu = vals[order[0]]
    mu = np.sqrt(nu)
    if mu.real < 0:
        mu = -mu
    full = np.zeros(shape, dtype=np.complex128)
    full[even] = vecs[:, order[0]]
    full = full + hop_c(U, full, parity=1) / mu
    return mu, vals[order], full, count[0]


def main(name):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import get_config, random_su3_links
    cfg = get_config(name)
    dims = cfg["dims"]
    U = random_su3_links(dims, cfg["eps"], cfg["link_seed"])
    from .wilson import hop
    t0 = time.time()
    tol, ncv = 1e-5, 250
    mu_c, vals, v, nmv = rightmost_eig_eo(U, dims, tol=tol, ncv=ncv, progress=500, k=1)
    resid = float(np.linalg.norm(hop(U, v) - mu_c * v) / (abs(mu_c) * np.linalg.norm(v)))
    mu = float(mu_c.real)
    vals = np.array([mu_c])
    delta = cfg.get("delta", 1e-3)
    out = dict(config=name, dims=list(dims), eps=cfg["eps"], link_seed=cfg["link_seed"],
               rightmost_mu=[[float(v.real), float(v.imag)] for v in vals],
               max_re_mu=mu, eig_resid=resid, delta=delta, kappa=(1.0 - delta) / mu, matvecs=nmv,
               seconds=time.time() - t0,
               method="ARPACK eigs(which='LR', k=1, ncv=%d, tol=%g) on the even/odd square D_eo D_oe "
                      "of the oracle hop; mu = sqrt of its rightmost eigenvalue" % (ncv, tol))
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "synth",
                        "%s_kappa.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c3")
