"""The C header compiles as C99 and a plain C caller links against the
in-tree library and the HIP runtime (no GPU needed): the program that
tests/test_gpu_c_client.py runs on the GPU, built here into a scratch folder
with every gcc warning enabled."""
import importlib.util
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("c_client_build",
                                               os.path.join(HERE, "c_abi", "build.py"))
client_build = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(client_build)


def test_c_client_compiles_and_links_without_warnings(tmp_path):
    out = str(tmp_path / "trace_client")
    r = subprocess.run(client_build.command(out), capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "warning" not in r.stderr, r.stderr
    assert os.access(out, os.X_OK)
