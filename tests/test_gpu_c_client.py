"""The library called from plain C (tests/c_abi/trace_client.c): the C99
program sets up the field of view with rr_fov_directions (Sec. III E), builds
the vertex tensor (Eq. tidalexample, Sec. III H) and traces every ray
(Eqs. sumIc, Iclensing) with device memory from the HIP runtime.  Its kappa,
Kahan compensation, crossing hashes, counts and status equal, bit for bit,
those of the same calls made through the Python binding, and its crossing
hashes equal the FP64 oracle's."""
import math
import os
import subprocess

import numpy as np
import pytest

from paper_1601_02012_amd import inputs as I

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CLIENT = os.path.join(HERE, "c_abi", "trace_client")


def _read(path, prec):
    with open(path, "rb") as f:
        nr = int(np.frombuffer(f.read(8), np.int64)[0])
        assert int(np.frombuffer(f.read(4), np.int32)[0]) == prec
        kap = np.frombuffer(f.read(nr * (4 if prec else 8)), np.float32 if prec else np.float64)
        comp = np.frombuffer(f.read(nr * 4), np.float32) if prec else None
        h = np.frombuffer(f.read(nr * 8), np.uint64)
        c = np.frombuffer(f.read(nr * 8), np.int64)
        s = np.frombuffer(f.read(nr * 4), np.int32)
        assert f.read() == b""
    return kap, comp, h, c, s


@pytest.mark.parametrize("prec", [0, 1])
def test_c_caller_matches_the_binding_and_the_oracle(tmp_path, oracle, prec):
    import torch
    from paper_1601_02012_amd import api
    from tests._cases import hashes_u64
    assert os.access(CLIENT, os.X_OK), "tests/c_abi/trace_client is not built (run build())"
    n, box, nx, fov_deg, chis = 24, 96.0, 16, 3.0, 150.0
    rng = np.random.default_rng(31)
    phi = I.poisson_phi(I.gaussian_field(n, box, rng, slope=-2.0), box).astype(np.float64)
    phi_path = tmp_path / "phi.bin"
    phi.tofile(phi_path)
    out = tmp_path / "out.bin"
    cmd = [CLIENT, str(phi_path), str(n), repr(box), str(prec), repr(fov_deg), str(nx), repr(chis),
           str(out)]
    print("running", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "refused as expected" in r.stdout
    kap, comp, h, c, s = _read(out, prec)
    assert np.all(s == 0)

    # the same calls through the binding
    fov = fov_deg * (math.pi / 180.0)
    dirs = api.fov_directions((0.0, 0.0, 1.0), fov, fov, nx, nx)
    p = phi.astype(np.float32) if prec else phi
    g = api.Grid(torch.as_tensor(p).cuda(), box)
    t = api.TidalTensor(g, "fp32" if prec else "fp64").build()
    plan = api.Plan()
    b = api.RayBundle(torch.as_tensor(dirs).cuda(), nx, nx, chis, chis, 0.0, 0,
                      (0.0, 0.0, 1.0), fov, fov)
    o = api.trace(plan, t, [b], (0.0, 0.0, 0.0), debug=True, persistent=0)
    torch.cuda.synchronize()
    assert o.kappa.cpu().numpy().tobytes() == kap.tobytes()
    if prec:
        assert o.kappa_comp.cpu().numpy().tobytes() == comp.tobytes()
    assert np.array_equal(hashes_u64(o.hash), h)
    assert np.array_equal(o.count.cpu().numpy(), c)
    t.close()
    plan.close()

    # and the oracle's crossing lists
    ref = oracle.trace_uniform(n, box, (0.0, 0.0, 0.0), dirs, chis, chis, 0.0,
                               phi=p.astype(np.float64))
    assert np.array_equal(h, ref.hash)
    assert np.array_equal(c, ref.ncross)
