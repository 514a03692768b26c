"""Shared set-up of GPU parity cases: the same seeded inputs go to the HIP
library (through the C ABI binding) and to the FP64 oracle."""
import math

import numpy as np

from paper_1601_02012_amd import inputs as I


def kappa_tolerance_ok(got, ref, rel=1e-5, abs_=1e-7):
    """|got - ref| <= max(rel |ref|, abs) for every ray."""
    err = np.abs(got - ref)
    lim = np.maximum(rel * np.abs(ref), abs_)
    return bool(np.all(err <= lim)), float(np.max(err / lim)) if err.size else 0.0


def gpu_grid(api, phi, box, boundary="periodic", dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(phi))
    if dtype is not None:
        t = t.to(dtype)
    return api.Grid(t.cuda(), box, boundary=boundary)


def gpu_bundle(api, dirs, nx, ny, chi_s, chi_hi, chi_lo, offset=0):
    import torch
    d = torch.as_tensor(np.ascontiguousarray(dirs, dtype=np.float64)).cuda()
    return api.RayBundle(d, nx, ny, chi_s, chi_hi, chi_lo, offset)


def hashes_u64(t):
    return t.cpu().numpy().view(np.uint64)


def small_periodic_case(seed=0, n=32, box=64.0, nx=37, ny=13, fov_deg=4.0, chi=(90.0, 80.0, 3.0)):
    rng = np.random.default_rng(seed)
    delta = I.gaussian_field(n, box, rng, slope=-2.0)
    phi = I.poisson_phi(delta, box)
    fov = math.radians(fov_deg)
    dirs = I.fov_directions((0.15, -0.1, 1.0), fov, fov * ny / nx, nx, ny)
    return phi, dirs
