"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *generates inputs*: base-material tensors and nodal
level-set fields (or per-element densities) on the periodic N^3 grid whose
nodes sit at (i, j, k) / N.  It contains none of the homogenisation
arithmetic: no smoothed Heaviside, no element matrices, no solve.  Both the
CPU oracle and the GPU path consume its output identically.

Conventions
-----------
* node index n = i + N*(j + N*k), x fastest; arrays are returned flat in that
  order (length N^3), float64.
* level set sign follows Sec. 2.1 of the paper: phi < 0 is solid, phi > 0 void.
* element (i, j, k) spans nodes (i..i+1, j..j+1, k..k+1) modulo N; element
  arrays use the same flat order as nodes.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Material", "material_workload", "material_pzt5a", "node_coords",
    "sphere_levelset", "grf_levelset", "gyroid_levelset", "paper_levelset",
    "laminate_density", "random_density",
]


class Material:
    """Base-material tensors in SI units, Voigt order (xx, yy, zz, yz, xz, xy).

    C : (6, 6) Pa, elasticity at fixed electric field.
    e : (3, 6) C/m^2, piezoelectric stress coefficients.
    kappa : (3, 3) F/m, permittivity at fixed strain.
    void_scale : ersatz scale applied to all three tensors in void.
    """

    def __init__(self, C, e, kappa, void_scale=1e-3):
        self.C = np.array(C, dtype=np.float64).reshape(6, 6)
        self.e = np.array(e, dtype=np.float64).reshape(3, 6)
        self.kappa = np.array(kappa, dtype=np.float64).reshape(3, 3)
        self.void_scale = float(void_scale)

    def flat(self):
        return (self.C.ravel().copy(), self.e.ravel().copy(),
                self.kappa.ravel().copy(), self.void_scale)


def _ti_material(c11, c12, c13, c33, c44, c66, e31, e33, e15, k11, k33, void_scale):
    C = np.zeros((6, 6))
    C[0, 0] = C[1, 1] = c11
    C[0, 1] = C[1, 0] = c12
    C[0, 2] = C[2, 0] = C[1, 2] = C[2, 1] = c13
    C[2, 2] = c33
    C[3, 3] = C[4, 4] = c44
    C[5, 5] = c66
    e = np.zeros((3, 6))
    e[2, 0] = e[2, 1] = e31
    e[2, 2] = e33
    e[0, 4] = e[1, 3] = e15
    kap = np.diag([k11, k11, k33])
    return Material(C, e, kap, void_scale)


def material_workload(void_scale=1e-3):
    """Transversely isotropic PZT-like base material used by every workload.

    C11=120.3, C12=75.2, C13=75.1, C33=110.9, C44=21.1, C66=22.6 GPa;
    e31=-5.4, e33=15.8, e15=12.3 C/m^2; kappa11=8.11e-9, kappa33=7.35e-9 F/m.
    """
    g = 1e9
    return _ti_material(120.3 * g, 75.2 * g, 75.1 * g, 110.9 * g, 21.1 * g, 22.6 * g,
                        -5.4, 15.8, 12.3, 8.11e-9, 7.35e-9, void_scale)


def material_pzt5a(void_scale=1e-3):
    """z-poled PZT-5A exactly as printed in Sec. 2.3 of the paper."""
    t = 1e10
    return _ti_material(12.04 * t, 7.52 * t, 7.51 * t, 11.09 * t, 2.1 * t, 2.3 * t,
                        -5.4, 15.8, 12.3, 4.78e-9, 7.35e-9, void_scale)


def node_coords(n):
    """Node coordinates (x, y, z), each flat of length n^3, x fastest."""
    g = np.arange(n, dtype=np.float64) / n
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def sphere_levelset(n, radius=0.3):
    """Void sphere of the given radius at the cell centre, exact signed distance.

    phi = radius - |x - c| is positive (void) inside the sphere.
    """
    x, y, z = node_coords(n)
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2)
    return radius - r


def _grf_modes(seed, corr_len, kmax):
    """Fixed mode set and complex normal coefficients of a periodic Gaussian field."""
    ks = np.arange(-kmax, kmax + 1)
    kx, ky, kz = np.meshgrid(ks, ks, ks, indexing="ij")
    k2 = (2.0 * np.pi) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2)
    amp = np.exp(-corr_len ** 2 * k2 / 4.0)
    rng = np.random.default_rng(seed)
    shape = amp.shape
    coef = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    var = np.sum(amp ** 2)
    gvar = np.sum(amp ** 2 * k2)
    return ks, coef * amp / np.sqrt(var), np.sqrt(gvar / var)


def _eval_modes(n, ks, coef):
    """Real part of sum_k coef_k exp(2 pi i k.x) on the n^3 node grid (separable)."""
    g = np.arange(n, dtype=np.float64) / n
    E = np.exp(2j * np.pi * np.outer(ks, g))          # (nk, n)
    # f[kz, ky, kx] with x fastest at the end
    t = np.einsum("abc,cz->abz", coef, E)              # contract kz -> z
    t = np.einsum("abz,by->ayz", t, E)                 # contract ky -> y
    t = np.einsum("ayz,ax->zyx", t, E)                 # contract kx -> x
    return t.real.ravel()


def grf_levelset(n, seed=2410, corr_len=0.1, solid_fraction=0.5, kmax=12):
    """Periodic Gaussian random field level set (resolution independent).

    Gaussian covariance exp(-r^2 / 2 l^2) by spectral synthesis over the modes
    |k_i| <= kmax (the amplitude filter is below 1e-6 beyond), unit variance.
    The threshold t is the solid_fraction quantile of the nodal values, so that
    that fraction of nodes is solid (phi < 0).  phi = (f - t) / RMS|grad f|,
    which makes the interface band about as wide in elements as a distance.
    """
    ks, coef, grad_rms = _grf_modes(seed, corr_len, kmax)
    f = _eval_modes(n, ks, coef)
    t = np.quantile(f, solid_fraction)
    return (f - t) / grad_rms


def gyroid_levelset(n, seed=2411, noise=0.05):
    """Gyroid-like triply periodic field with uniform nodal noise.

    g = cos2pi x sin2pi y + cos2pi y sin2pi z + cos2pi z sin2pi x + U(-noise, noise),
    phi = g / RMS|grad g_smooth| with RMS|grad g_smooth| = 2 pi sqrt(3/2).
    """
    x, y, z = node_coords(n)
    tp = 2.0 * np.pi
    g = (np.cos(tp * x) * np.sin(tp * y) + np.cos(tp * y) * np.sin(tp * z)
         + np.cos(tp * z) * np.sin(tp * x))
    rng = np.random.default_rng(seed)
    g = g + rng.uniform(-noise, noise, size=g.shape)
    return g / (tp * np.sqrt(1.5))


def paper_levelset(n):
    """The weak-scaling test geometry of Sec. 2.5.4: phi = -prod cos(2 pi x_i) - 0.2.

    Scaled by its RMS gradient 2 pi sqrt(3/8) so the smoothing band is about
    as wide as for a distance function.
    """
    x, y, z = node_coords(n)
    tp = 2.0 * np.pi
    f = -np.cos(tp * x) * np.cos(tp * y) * np.cos(tp * z) - 0.2
    return f / (tp * np.sqrt(3.0 / 8.0))


def laminate_density(n, axis=2, seed=7, profile="random"):
    """Per-element density depending only on the element layer along `axis`.

    profile "random": layer densities U(0, 1) from default_rng(seed) with the
    first two layers forced to 1 and 0; "half": solid in the first n/2 layers.
    """
    if profile == "half":
        layer = (np.arange(n) < n // 2).astype(np.float64)
    else:
        rng = np.random.default_rng(seed)
        layer = rng.uniform(0.0, 1.0, size=n)
        layer[0] = 1.0
        if n > 1:
            layer[1] = 0.0
    idx = np.arange(n)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    which = (i, j, k)[axis].ravel()
    return layer[which].copy()


def random_density(n, seed=11, low=0.0, high=1.0):
    """Independent U(low, high) per-element densities."""
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=n ** 3)
