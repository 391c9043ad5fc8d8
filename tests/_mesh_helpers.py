"""Small shared fixtures for the CPU tests (mesh + fields on tiny lattices)."""
import numpy as np

from paper_2101_09059_amd import inputs
from oracle import element, assembly


def tiny_case(n_theta=10, n_z=6, S=2, seed=0, nu=0.49, k=5.0 / 6.0):
    m = inputs.cylinder(1.0, 4.0, n_theta, n_z)
    kh, A, _ = element.reference_stiffness(m.xyz, m.tri, nu, k)
    rng = np.random.default_rng(seed)
    eh = 7e5 * np.exp(0.2 * rng.standard_normal((m.n_el, S)))
    h = 0.1 * np.exp(0.2 * rng.standard_normal((m.n_el, S)))
    return m, kh, A, eh, h


def free_system(m, kh, A, eh_col, h_col, rho=1.0):
    K = assembly.assemble_stiffness(m.tri, kh, eh_col, m.n_nodes)
    mn = assembly.lumped_mass(m.tri, A, h_col, rho, m.n_nodes)
    free = ~m.fixed.reshape(-1).astype(bool)
    return K, mn, free
