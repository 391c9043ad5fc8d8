"""Pins for the oracle's per-sample assembly and lumped mass."""
import numpy as np

from oracle import assembly
from tests._mesh_helpers import tiny_case


def test_symmetry_and_reciprocity():
    m, kh, A, eh, h = tiny_case()
    K = assembly.assemble_stiffness(m.tri, kh, eh[:, 0], m.n_nodes)
    assert abs(K - K.T).max() <= 1e-13 * abs(K).max()
    rng = np.random.default_rng(4)
    u, v = rng.normal(size=(2, m.n_dof))
    assert np.isclose(u @ (K @ v), v @ (K @ u), rtol=1e-13)


def test_translation_null_space_of_unclamped_matrix():
    m, kh, A, eh, h = tiny_case()
    K = assembly.assemble_stiffness(m.tri, kh, eh[:, 1], m.n_nodes)
    for c in range(3):
        t = np.zeros(m.n_dof)
        t[c::3] = 1.0
        assert np.linalg.norm(K @ t) <= 1e-12 * abs(K).max()


def test_element_by_element_product_matches_csr():
    # scattering Eh_e Khat_e u_e element by element equals the assembled K u
    m, kh, A, eh, h = tiny_case()
    rng = np.random.default_rng(5)
    u = rng.normal(size=m.n_dof)
    K = assembly.assemble_stiffness(m.tri, kh, eh[:, 0], m.n_nodes)
    r = np.zeros(m.n_dof)
    for e in range(m.n_el):
        d = (3 * m.tri[e][:, None] + np.arange(3)).reshape(-1)
        r[d] += eh[e, 0] * kh[e] @ u[d]
    assert np.allclose(r, K @ u, rtol=0, atol=1e-12 * np.abs(r).max())


def test_lumped_mass_total():
    # total mass of the lumped matrix is rho * sum_e h_e A_e, and the
    # cylinder's lateral area is 2 R sin(pi/n) n L on the faceted mesh
    m, kh, A, eh, h = tiny_case()
    hc = np.full(m.n_el, 0.1)
    mn = assembly.lumped_mass(m.tri, A, hc, 2.0, m.n_nodes)
    lateral = 2.0 * np.sin(np.pi / m.n_theta) * m.n_theta * m.length
    assert np.isclose(mn.sum(), 2.0 * 0.1 * lateral, rtol=1e-13)
