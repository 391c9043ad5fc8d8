"""Seeded synthetic inputs for the ensemble wall solver.

This module builds the things the solver is *given*: wall meshes, the
per-element / per-sample material fields, the nodal traction load vector,
the clamped dofs and the per-node radial directions.  It holds none of the
solver's own arithmetic (no element matrices, no assembly, no time
stepping), so both the HIP library and the CPU oracle can consume the same
inputs without sharing any solver code.

Stand-ins (the paper's own meshes, fluid tractions and waveforms are not
available):
  * meshes are analytic tubes (straight clamped cylinder, curved tapered
    tube, a seeded batch of straight tubes) triangulated on a structured
    (theta, axial) node lattice;
  * the nodal load is the lumped wall traction of an analytic pressure
    field (optionally tapered along the axis, plus a seeded tangential
    shear), in place of the fluid solver's wall stress (Sec. 2.2.3);
  * the log-modulus and log-thickness fields are Gaussian with Matern
    covariance (Sec. 2.1); for lattices too large for a dense Cholesky they
    are sampled exactly on the nodes by circulant embedding of the Matern
    covariance on the periodic-theta lattice, then interpolated linearly to
    the element centroids.

Units are cgs throughout (cm, g, s, dyn/cm^2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy import special

__all__ = [
    "Mesh", "cylinder", "curved_tube", "tube_batch_specs", "lognormal_fields_device",
    "matern_nodal_lattice", "centroid_average", "lognormal_fields",
    "traction_load", "CONFIGS",
]


@dataclasses.dataclass
class Mesh:
    """Triangulated lumen surface.

    xyz     [n_nodes, 3] float64 node coordinates (cm)
    tri     [n_el, 3]    int32 node indices, counter-clockwise seen from
                         outside, so (p2-p1) x (p3-p1) points outward
    fixed   [n_nodes, 3] uint8, 1 where the dof is clamped
    radial  [n_nodes, 3] float64 unit outward radial direction per node
    axial   [n_nodes]    float64 arc length of the closest centreline point
    length  float        centreline length L
    n_theta, n_z         lattice shape (node (i, j) has index i + j*n_theta)
    """
    xyz: np.ndarray
    tri: np.ndarray
    fixed: np.ndarray
    radial: np.ndarray
    axial: np.ndarray
    length: float
    n_theta: int
    n_z: int
    name: str = "mesh"

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_el(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes


def _lattice_triangles(n_theta: int, n_z: int) -> np.ndarray:
    """Split every lattice quad along its (i,j)-(i+1,j+1) diagonal."""
    i = np.arange(n_theta)
    j = np.arange(n_z - 1)
    I, J = np.meshgrid(i, j, indexing="xy")        # [n_z-1, n_theta]
    n00 = I + J * n_theta
    n10 = (I + 1) % n_theta + J * n_theta
    n01 = I + (J + 1) * n_theta
    n11 = (I + 1) % n_theta + (J + 1) * n_theta
    t_a = np.stack([n00, n10, n11], axis=-1).reshape(-1, 3)
    t_b = np.stack([n00, n11, n01], axis=-1).reshape(-1, 3)
    # interleave so the two triangles of one quad are adjacent in memory
    tri = np.empty((t_a.shape[0] * 2, 3), dtype=np.int32)
    tri[0::2] = t_a
    tri[1::2] = t_b
    return tri


def _clamp_end_rings(n_theta: int, n_z: int) -> np.ndarray:
    fixed = np.zeros((n_theta * n_z, 3), dtype=np.uint8)
    fixed[:n_theta] = 1
    fixed[(n_z - 1) * n_theta:] = 1
    return fixed


def cylinder(R: float, L: float, n_theta: int, n_z: int) -> Mesh:
    """Straight cylinder, node (i, j) at (R cos t_i, R sin t_i, z_j),
    t_i = 2 pi i / n_theta, z_j = j L / (n_z - 1); both end rings clamped
    in all three translations (fully fixed ends, Sec. 3.1)."""
    th = 2.0 * np.pi * np.arange(n_theta) / n_theta
    z = np.arange(n_z) * (L / (n_z - 1))
    TH, Z = np.meshgrid(th, z, indexing="xy")      # [n_z, n_theta]
    xyz = np.stack([R * np.cos(TH), R * np.sin(TH), Z], axis=-1).reshape(-1, 3)
    radial = np.stack([np.cos(TH), np.sin(TH), np.zeros_like(TH)], axis=-1).reshape(-1, 3)
    return Mesh(xyz=np.ascontiguousarray(xyz), tri=_lattice_triangles(n_theta, n_z),
                fixed=_clamp_end_rings(n_theta, n_z), radial=np.ascontiguousarray(radial),
                axial=Z.reshape(-1).copy(), length=float(L), n_theta=n_theta, n_z=n_z,
                name=f"cylinder_R{R}_L{L}_{n_theta}x{n_z}")


def curved_tube(n_theta: int, n_z: int, arc_radius: float = 8.0, length: float = 20.0,
                r_in: float = 1.2, r_out: float = 0.6) -> Mesh:
    """Curved tapered tube: the centreline is a planar arc of radius
    `arc_radius` and arc length `length`; the lumen radius falls linearly
    from r_in to r_out along it; the binormal is constant.  Node (i, j) sits
    at c(s_j) + r(s_j) (cos t_i n(s_j) + sin t_i b)."""
    th = 2.0 * np.pi * np.arange(n_theta) / n_theta
    s = np.arange(n_z) * (length / (n_z - 1))
    phi = s / arc_radius
    c = np.stack([arc_radius * (1.0 - np.cos(phi)), np.zeros_like(phi), arc_radius * np.sin(phi)], -1)
    nrm = np.stack([np.cos(phi), np.zeros_like(phi), -np.sin(phi)], -1)
    b = np.array([0.0, 1.0, 0.0])
    r = r_in + (r_out - r_in) * s / length
    er = np.cos(th)[None, :, None] * nrm[:, None, :] + np.sin(th)[None, :, None] * b[None, None, :]
    xyz = c[:, None, :] + r[:, None, None] * er                  # [n_z, n_theta, 3]
    return Mesh(xyz=np.ascontiguousarray(xyz.reshape(-1, 3)), tri=_lattice_triangles(n_theta, n_z),
                fixed=_clamp_end_rings(n_theta, n_z),
                radial=np.ascontiguousarray(er.reshape(-1, 3)),
                axial=np.repeat(s, n_theta), length=float(length), n_theta=n_theta, n_z=n_z,
                name=f"curved_tube_{n_theta}x{n_z}")


def tube_batch_specs(seed: int, count: int = 16):
    """Uneven batch of straight tubes: node count log-uniform in [5e3, 4e5],
    radius U(0.3, 1.5) cm, length U(5, 25) cm, ensemble width
    32*round(exp(U[ln 32, ln 512])/32).  n_theta = max(8, round(sqrt(n 2 pi R / L)))
    keeps the lattice cells near square."""
    rng = np.random.default_rng(seed)
    specs = []
    for _ in range(count):
        n = math.exp(rng.uniform(math.log(5e3), math.log(4e5)))
        R = rng.uniform(0.3, 1.5)
        L = rng.uniform(5.0, 25.0)
        S = int(32 * round(math.exp(rng.uniform(math.log(32), math.log(512))) / 32))
        S = max(32, S)
        n_theta = max(8, int(round(math.sqrt(n * 2.0 * math.pi * R / L))))
        n_z = max(3, int(round(n / n_theta)))
        specs.append(dict(R=R, L=L, n_theta=n_theta, n_z=n_z, S=S))
    return specs


# ---------------------------------------------------------------------------
# Random fields
# ---------------------------------------------------------------------------

def _matern(d: np.ndarray, sigma: float, nu: float, kappa: float) -> np.ndarray:
    """Matern covariance (Sec. 2.1) evaluated on distances d."""
    x = kappa * np.asarray(d, dtype=np.float64)
    out = np.full_like(x, sigma * sigma)
    pos = x > 0
    xp = x[pos]
    out[pos] = sigma * sigma * (2.0 ** (1.0 - nu) / special.gamma(nu)) * xp ** nu * special.kv(nu, xp)
    return out


def matern_nodal_lattice(mesh: Mesh, n_samples: int, rng: np.random.Generator,
                         sigma: float, rho: float, nu: float = 1.0,
                         radius: Optional[float] = None) -> np.ndarray:
    """Zero-mean Gaussian samples [n_nodes, n_samples] with Matern covariance
    of the chord distance between lattice nodes of a straight cylinder,
    d^2 = 2 R^2 (1 - cos dtheta) + dz^2, by circulant embedding (periodic in
    theta, zero-padded to period >= 2 (n_z - 1) along the axis).  For
    non-cylindrical tubes pass `radius` (a representative radius); the
    lattice spacing along the axis is taken from the centreline length."""
    nt, nz = mesh.n_theta, mesh.n_z
    if radius is None:
        R = float(np.mean(np.linalg.norm(mesh.xyz[:nt, :2], axis=1)))
    else:
        R = float(radius)
    dz = mesh.length / (nz - 1)
    kappa = math.sqrt(8.0 * nu) / rho
    mz = 1
    while mz < 2 * (nz - 1):
        mz *= 2
    kz = np.arange(mz)
    lagz = np.minimum(kz, mz - kz) * dz
    kt = np.arange(nt)
    dth = 2.0 * np.pi * kt / nt
    chord2 = 2.0 * R * R * (1.0 - np.cos(dth))
    D = np.sqrt(chord2[None, :] + lagz[:, None] ** 2)            # [mz, nt]
    c = _matern(D, sigma, nu, kappa)
    lam = np.fft.fft2(c).real
    lam = np.maximum(lam, 0.0)
    scale = np.sqrt(lam / (mz * nt))
    out = np.empty((n_samples, nz * nt), dtype=np.float64)
    batch = 16
    k = 0
    while k < n_samples:
        b = min(batch, (n_samples - k + 1) // 2)
        z = rng.standard_normal((b, mz, nt)) + 1j * rng.standard_normal((b, mz, nt))
        f = np.fft.fft2(scale[None] * z, axes=(1, 2))[:, :nz, :].reshape(b, -1)
        for i in range(b):
            if k < n_samples:
                out[k] = f[i].real
                k += 1
            if k < n_samples:
                out[k] = f[i].imag
                k += 1
    return np.ascontiguousarray(out.T)


def _lattice_spectrum(mesh: Mesh, sigma: float, rho: float, nu: float, radius: Optional[float]):
    """Square root of the circulant embedding's eigenvalues, scaled for a
    size-(mz, nt) FFT, as used by matern_nodal_lattice."""
    nt, nz = mesh.n_theta, mesh.n_z
    R = float(np.mean(np.linalg.norm(mesh.xyz[:nt, :2], axis=1))) if radius is None else float(radius)
    dz = mesh.length / (nz - 1)
    kappa = math.sqrt(8.0 * nu) / rho
    mz = 1
    while mz < 2 * (nz - 1):
        mz *= 2
    kz = np.arange(mz)
    lagz = np.minimum(kz, mz - kz) * dz
    dth = 2.0 * np.pi * np.arange(nt) / nt
    D = np.sqrt((2.0 * R * R * (1.0 - np.cos(dth)))[None, :] + lagz[:, None] ** 2)
    lam = np.maximum(np.fft.fft2(_matern(D, sigma, nu, kappa)).real, 0.0)
    return np.sqrt(lam / (mz * nt)), mz


def lognormal_fields_device(mesh: Mesh, S: int, seed: int, E_mean: float = 7.0e6, h_mean: float = 0.1,
                            sigma_log: float = 0.2, rho: float = 2.0, nu: float = 1.0,
                            radius: Optional[float] = None, device: str = "cuda"):
    """lognormal_fields for large lattices, drawn with torch on `device`:
    the same circulant-embedding construction (each complex FFT gives two
    independent fields, real and imaginary parts), with torch's seeded
    generator instead of numpy's, so the draws differ from lognormal_fields
    but follow the same distribution.  Returns float64 numpy (E h), h
    [n_el, S]."""
    import torch
    nt, nz = mesh.n_theta, mesh.n_z
    scale_np, mz = _lattice_spectrum(mesh, sigma_log, rho, nu, radius)
    scale = torch.as_tensor(scale_np, dtype=torch.float64, device=device)
    tri = torch.as_tensor(mesh.tri.astype(np.int64), device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    out = []
    for mean in (E_mean, h_mean):
        cols = []
        k = 0
        while k < S:
            b = min(8, (S - k + 1) // 2)
            z = torch.complex(torch.randn((b, mz, nt), generator=gen, device=device, dtype=torch.float64),
                              torch.randn((b, mz, nt), generator=gen, device=device, dtype=torch.float64))
            f = torch.fft.fft2(scale[None] * z)[:, :nz, :].reshape(b, -1)
            g = torch.stack([f.real, f.imag], 1).reshape(2 * b, -1)[: S - k]      # [fields, n_nodes]
            cent = (g[:, tri[:, 0]] + g[:, tri[:, 1]] + g[:, tri[:, 2]]) / 3.0     # [fields, n_el]
            cols.append(torch.exp(math.log(mean) + cent).t().cpu())
            k += g.shape[0]
            del z, f, g, cent
        out.append(torch.cat(cols, 1).numpy())
    E, h = out
    np.multiply(E, h, out=E)
    return np.ascontiguousarray(E), np.ascontiguousarray(h)


def centroid_average(mesh: Mesh, nodal: np.ndarray) -> np.ndarray:
    """Value of the piecewise-linear interpolant at each element centroid."""
    t = mesh.tri
    return (nodal[t[:, 0]] + nodal[t[:, 1]] + nodal[t[:, 2]]) / 3.0


def lognormal_fields(mesh: Mesh, S: int, seed: int, E_mean: float = 7.0e6, h_mean: float = 0.1,
                     sigma_log: float = 0.2, rho: float = 2.0, nu: float = 1.0,
                     radius: Optional[float] = None):
    """Per-element, per-sample (E h) and h [n_el, S] float64 for the lattice
    meshes: log E and log h are independent Matern Gaussian fields with the
    given log-means and log-std, interpolated to the centroids."""
    rng = np.random.default_rng(seed)
    gE = centroid_average(mesh, matern_nodal_lattice(mesh, S, rng, sigma_log, rho, nu, radius))
    gh = centroid_average(mesh, matern_nodal_lattice(mesh, S, rng, sigma_log, rho, nu, radius))
    E = np.exp(math.log(E_mean) + gE)
    h = np.exp(math.log(h_mean) + gh)
    return np.ascontiguousarray(E * h), np.ascontiguousarray(h)


# ---------------------------------------------------------------------------
# Wall traction (stand-in for the fluid solver's wall stress)
# ---------------------------------------------------------------------------

def traction_load(mesh: Mesh, p0: float, axial_taper: float = 0.0, shear_frac: float = 0.0,
                  seed: Optional[int] = None) -> np.ndarray:
    """Nodal force [n_nodes, 3]: outward pressure p(x) = p0 (1 - taper x / L)
    at each element centroid, times the element normal, lumped A_e/3 to each
    node; plus, if shear_frac > 0, a seeded random unit tangent per element
    of magnitude shear_frac * p0 lumped the same way.  Clamped dofs carry
    their load too; the solver ignores loads on clamped dofs."""
    t = mesh.tri
    p1, p2, p3 = mesh.xyz[t[:, 0]], mesh.xyz[t[:, 1]], mesh.xyz[t[:, 2]]
    cr = np.cross(p2 - p1, p3 - p1)
    twoA = np.linalg.norm(cr, axis=1)
    n = cr / twoA[:, None]
    A = 0.5 * twoA
    x = (mesh.axial[t[:, 0]] + mesh.axial[t[:, 1]] + mesh.axial[t[:, 2]]) / 3.0
    p = p0 * (1.0 - axial_taper * x / mesh.length)
    fe = (p * A / 3.0)[:, None] * n
    if shear_frac > 0.0:
        rng = np.random.default_rng(seed)
        g = rng.standard_normal((t.shape[0], 3))
        g -= np.sum(g * n, axis=1)[:, None] * n
        g /= np.linalg.norm(g, axis=1)[:, None]
        fe = fe + (shear_frac * p0 * A / 3.0)[:, None] * g
    F = np.zeros((mesh.n_nodes, 3))
    for a in range(3):
        np.add.at(F, t[:, a], fe)
    return F


# ---------------------------------------------------------------------------
# Workload definitions (sizes, value distributions, seeds)
# ---------------------------------------------------------------------------

CONFIGS = {
    # plain FP64, tiny: 40 x 20 node cylinder, S = 8, ramp 0.05 s, 2,000 steps
    "c1_tiny": dict(R=1.0, L=10.0, n_theta=40, n_z=20, S=8, seed=1, p0=1.33e5,
                    ramp="sine", T_ramp=0.05, steps=2000, nu=0.49, shear_k=5.0 / 6.0,
                    rho=1.0, alpha=50.0, safety=0.9, field="dense_cholesky"),
    # plain method at scale: 400 x 500 node cylinder, S = 256, steady load, 20,000 steps
    "c2_cylinder": dict(R=1.0, L=10.0, n_theta=400, n_z=500, S=256, seed=2, p0=1.33e5,
                        ramp="step", T_ramp=0.0, steps=20000, nu=0.49, shear_k=5.0 / 6.0,
                        rho=1.0, alpha=50.0, safety=0.9, field="circulant"),
    # precision form: curved tapered tube, 500 x 2,000 nodes, S = 1,024, pulsatile + shear
    "c3_curved": dict(n_theta=500, n_z=2000, S=1024, seed=3, p0=1.33e5, ramp="sine_pulse",
                      T_ramp=0.05, period=1.0, pulse_amp=0.3, axial_taper=0.2, shear_frac=0.01,
                      steps=100000, nu=0.49, shear_k=5.0 / 6.0, rho=1.0, alpha=50.0, safety=0.9,
                      field="circulant"),
    # batching form: 16 uneven tubes, seeded sizes and widths, steady load
    "c4_batch": dict(count=16, seed=4, p0=1.33e5, ramp="step", steps=10000, nu=0.49,
                     shear_k=5.0 / 6.0, rho=1.0, alpha=50.0, safety=0.9, field="circulant"),
}


# ---------------------------------------------------------------------------
# Karhunen-Loeve expansion of the nodal Matern field on a cylinder lattice
# ---------------------------------------------------------------------------

def cylinder_kl_basis(mesh: Mesh, n_modes: int, sigma: float, rho: float, nu: float = 1.0,
                      radius: Optional[float] = None):
    """Leading eigenpairs of the nodal covariance (Matern of the chord
    distance, as in matern_nodal_lattice) on the periodic-theta lattice.

    The covariance is block-circulant in theta, so it splits exactly per
    azimuthal wave number m into symmetric Toeplitz blocks along the axis,
    T_m(dz) = sum_k c(theta_k, dz) cos(2 pi m k / n_theta); their
    eigenvectors v give nodal modes w_m(theta_i) v(z_j) with w_0 = n^-1/2,
    cos / sin pairs sqrt(2/n) cos(m theta), sqrt(2/n) sin(m theta) for
    0 < m < n/2.  Returns (lam [n_modes] descending, phi [n_nodes, n_modes]
    orthonormal over the nodes, captured fraction of the total variance)."""
    from scipy import linalg

    nt, nz = mesh.n_theta, mesh.n_z
    R = float(np.mean(np.linalg.norm(mesh.xyz[:nt, :2], axis=1))) if radius is None else float(radius)
    dz = mesh.length / (nz - 1)
    kappa = math.sqrt(8.0 * nu) / rho
    th = 2.0 * np.pi * np.arange(nt) / nt
    chord2 = 2.0 * R * R * (1.0 - np.cos(th))
    lag = np.arange(nz) * dz
    c = _matern(np.sqrt(chord2[None, :] + lag[:, None] ** 2), sigma, nu, kappa)   # [nz, nt]
    spec = np.fft.fft(c, axis=1).real                                              # T_m(dz) per m
    cands = []  # (lam, m, kind, v)
    kth = None
    for m in range(nt // 2 + 1):
        col = spec[:, m]
        if kth is not None and col[0] * nz < kth * 1e-3:
            break
        w, V = linalg.eigh(linalg.toeplitz(col))
        order = np.argsort(w)[::-1][:n_modes]
        kinds = ("c",) if (m == 0 or 2 * m == nt) else ("c", "s")
        for idx in order:
            for kd in kinds:
                cands.append((float(w[idx]), m, kd, V[:, idx]))
        cands.sort(key=lambda t: -t[0])
        cands = cands[:n_modes]
        if len(cands) == n_modes:
            kth = cands[-1][0]
            if w.max() < kth:
                break
    lam = np.array([t[0] for t in cands])
    phi = np.empty((nt * nz, len(cands)))
    ii = np.arange(nt)
    for k, (_, m, kd, v) in enumerate(cands):
        if m == 0:
            w_t = np.full(nt, 1.0 / math.sqrt(nt))
        elif 2 * m == nt:
            w_t = np.cos(np.pi * ii) / math.sqrt(nt)
        elif kd == "c":
            w_t = math.sqrt(2.0 / nt) * np.cos(2.0 * np.pi * m * ii / nt)
        else:
            w_t = math.sqrt(2.0 / nt) * np.sin(2.0 * np.pi * m * ii / nt)
        phi[:, k] = (v[:, None] * w_t[None, :]).reshape(-1)
    captured = float(lam.sum() / (nt * nz * sigma * sigma))
    return lam, phi, captured


def kl_fields(mesh: Mesh, lam: np.ndarray, phi: np.ndarray, xi_E: np.ndarray, xi_h: np.ndarray,
              E_mean: float = 7.0e6, h_mean: float = 0.1):
    """(E h) and h [n_el, S] from KL coefficients xi_E, xi_h [S, n_modes]:
    log-fields phi (sqrt(lam) xi) at the nodes, interpolated to centroids."""
    s = np.sqrt(lam)[None, :]
    gE = centroid_average(mesh, phi @ (s * xi_E).T)
    gh = centroid_average(mesh, phi @ (s * xi_h).T)
    E = np.exp(math.log(E_mean) + gE)
    h = np.exp(math.log(h_mean) + gh)
    return np.ascontiguousarray(E * h), np.ascontiguousarray(h)


CONFIGS["c5_learned"] = dict(R=1.0, L=10.0, n_theta=400, n_z=500, n_modes=64, p0=1.33e5, ramp="sine_pulse",
                             T_ramp=0.02, period=1.0, pulse_amp=0.3, window=0.03, nu=0.49, shear_k=5.0 / 6.0,
                             rho=1.0, alpha=50.0, safety=0.9, width=1024, n_hidden=3, n_train=4096,
                             n_hf=1024, n_lf=65536, n_ref=8192, epochs=600, batch=256, lr=1e-3,
                             weight_decay=3.0, val=0.1,
                             seeds=dict(train=5, hf=6, lf=7, ref=8, init=9))
