"""Checks of the seeded input generators (meshes, loads, KL basis)."""
import numpy as np

from oracle import matern
from paper_2101_09059_amd import inputs


def test_kl_basis_equals_dense_eigendecomposition():
    m = inputs.cylinder(1.0, 10.0, 24, 14)
    lam, phi, cap = inputs.cylinder_kl_basis(m, 20, 0.2, 2.0)
    d = np.linalg.norm(m.xyz[:, None, :] - m.xyz[None, :, :], axis=-1)
    C = matern.covariance(d, 0.2, 1.0, 2.0)
    w = np.linalg.eigvalsh(C)[::-1]
    assert np.allclose(lam, w[:20], rtol=1e-12, atol=1e-14 * w[0])
    assert np.allclose(phi.T @ phi, np.eye(20), atol=1e-12)
    assert np.abs(C @ phi - phi * lam).max() < 1e-12 * lam[0]
    assert abs(cap - w[:20].sum() / np.trace(C)) < 1e-12


def test_kl_fields_shapes_and_means():
    m = inputs.cylinder(1.0, 5.0, 16, 9)
    lam, phi, _ = inputs.cylinder_kl_basis(m, 8, 0.2, 2.0)
    rng = np.random.default_rng(0)
    eh, h = inputs.kl_fields(m, lam, phi, rng.standard_normal((2000, 8)), rng.standard_normal((2000, 8)))
    assert eh.shape == (m.n_el, 2000) and np.all(h > 0)
    assert abs(np.median(np.log(h)) - np.log(0.1)) < 0.02


def test_cylinder_mesh_orientation_and_clamps():
    m = inputs.cylinder(1.0, 4.0, 10, 6)
    p = m.xyz[m.tri]
    n = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    c = p.mean(axis=1)
    assert np.all(np.sum(n[:, :2] * c[:, :2], axis=1) > 0)       # normals point outward
    assert m.fixed[:10].all() and m.fixed[-10:].all() and not m.fixed[10:-10].any()
    F = inputs.traction_load(m, 2.0)
    # total pressure force on a closed ring vanishes
    assert np.abs(F.sum(axis=0)).max() < 1e-12 * np.abs(F).max() * m.n_nodes


def test_batch_specs_reproducible():
    a = inputs.tube_batch_specs(4)
    b = inputs.tube_batch_specs(4)
    assert a == b and len(a) == 16
    assert all(32 <= s["S"] <= 512 and s["S"] % 32 == 0 for s in a)
    # node counts log-uniform in [5e3, 4e5] up to the lattice rounding, and
    # the cells near square (ring spacing 2 pi R / n_theta against L / n_z)
    n = np.array([s["n_theta"] * s["n_z"] for s in a])
    assert n.min() >= 0.95 * 5e3 and n.max() <= 1.05 * 4e5
    aspect = np.array([(2 * np.pi * s["R"] / s["n_theta"]) / (s["L"] / (s["n_z"] - 1)) for s in a])
    assert np.all((aspect > 0.5) & (aspect < 2.0))


def test_device_fields_follow_the_lattice_distribution():
    """The torch-drawn fields (used for the 1M-node workload) have the
    distribution of the numpy ones: log-means, log-std and the correlation
    of neighbouring elements agree; the draw is reproducible by seed."""
    m = inputs.curved_tube(40, 100)
    eh, h = inputs.lognormal_fields_device(m, 64, 3, radius=0.9, device="cpu")
    eh2, h2 = inputs.lognormal_fields(m, 64, 3, radius=0.9)
    assert eh.shape == eh2.shape == (m.n_el, 64)
    for a, b in ((np.log(h), np.log(h2)), (np.log(eh / h), np.log(eh2 / h2))):
        assert abs(a.mean() - b.mean()) < 0.02
        assert abs(a.std() - b.std()) < 0.02
    c1 = np.corrcoef(np.log(h)[0], np.log(h)[1])[0, 1]
    c2 = np.corrcoef(np.log(h2)[0], np.log(h2)[1])[0, 1]
    assert abs(c1 - c2) < 0.05
    again, _ = inputs.lognormal_fields_device(m, 64, 3, radius=0.9, device="cpu")
    assert np.array_equal(again, eh)
