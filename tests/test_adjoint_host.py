"""The per-particle vector-Jacobian products of the adjoint (hat geometry,
stage derivative, deposited terms, wall reflection, Boris step), compiled
for the host and checked against central finite differences of the forward
functions they differentiate."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_vector_jacobian_products_match_finite_differences():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "adjoint_host_check")
        subprocess.run([hipcc, "-std=c++17", "-O1", "-o", exe, os.path.join(HERE, "adjoint_host_check.cpp")],
                       check=True, capture_output=True, cwd=d)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {l.split()[0]: float(l.split()[1]) for l in out.strip().splitlines()}
    assert len(res) == 17, res
    for name, err in res.items():
        assert err <= (5e-4 if name == "boris_step" else 1e-5), (name, err)
