"""Workload configurations (synthetic stand-ins for the paper's lattices).

Each entry names lattice extents (Lx, Ly, Lz, Lt), the link roughness eps,
hopping parameter(s) kappa, the number of Z(4) noise vectors and the Krylov
sizes: (m, k) for the reduced-system solves, (herm_m, herm_k) for the
full-lattice hermitian eigensolve that yields the n_hermitian modes (k must
exceed the number of wanted modes for the edge of a near-degenerate low
cluster to converge).  Seeds: links 1000 + config number, noise 2000 + config number.

The paper's own runs (Sec. 7-9) use 8^4 and 24^3x32 quenched beta=6.0
lattices and 16^3x48 dynamical ones with 200 Z(4) noises and
GMRES-DR(200,160); these stand-ins keep the lattice shapes and noise counts,
not the ensembles.
"""
import copy

CONFIGS = {
    # small case the oracle runs end to end in seconds
    "c1": dict(dims=(4, 4, 4, 4), eps=0.3, kappas=(0.12,), n_noise=8,
               m=20, k=10, pert_order=4, poly_degree=4, n_hermitian=10,
               herm_m=30, herm_k=15, link_seed=1001, noise_seed=2001),
    # plain FP64 method at 16^3x32
    "c2": dict(dims=(16, 16, 16, 32), eps=0.25, kappas=(0.120, 0.125, 0.128),
               n_noise=100, m=50, k=30, pert_order=7, poly_degree=7,
               n_hermitian=30, herm_m=80, herm_k=45, link_seed=1002, noise_seed=2002),
    # precision axis and headline throughput: 24^3x32 near-critical
    "c3": dict(dims=(24, 24, 24, 32), eps=0.2, kappas=None, delta=1e-3,
               n_noise=200, m=80, k=40, pert_order=7, poly_degree=7,
               n_hermitian=30, herm_m=80, herm_k=45, link_seed=1003, noise_seed=2003),
    # batching axis: several lattices, uneven right-hand-side counts
    "c4": dict(lattices=((8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32)),
               n_rhs=(17, 64, 160), eps=0.25, kappas=(0.125,), m=40, k=20,
               link_seed=1004, noise_seed=2004),
    # variance study (standard error vs deflated modes, relative efficiencies)
    # on the paper's small lattice shape, several configurations
    "c6": dict(dims=(8, 8, 8, 8), eps=0.25, kappas=(0.128,), n_noise=64, m=40, k=20,
               pert_order=7, poly_degree=7, n_hermitian=30, herm_m=80, herm_k=45,
               link_seed=1006, noise_seed=2006),
    # differentiation axis
    "c5": dict(dims=(12, 12, 12, 12), eps=0.25, kappas=(0.124,), n_noise=32,
               m=40, k=20, link_seed=1005, noise_seed=2005),
}


def get_config(name):
    return copy.deepcopy(CONFIGS[name])
