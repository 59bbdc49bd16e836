"""The library's host-side setup code under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU needed).

tests/host_sanitizer/driver.cpp is built with g++ together with the
library's host sources (reference element, mesh connectivity and geometry,
element orderings; none of them has device code or calls HIP) and run on
seeded meshes written here: a bounded and a periodic Kuhn cube, a general
(jittered, relabelled, renumbered) mesh and a periodic column.  It checks
the reference element of every order, builds each mesh at orders 1, 3 and
6, locates element centroids, and validates both orderings; the sanitizers
abort on any invalid memory access, leak or undefined behaviour.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2205_11052_amd", "csrc")


def _write_mesh(path, mesh):
    vxyz = np.ascontiguousarray(mesh["vxyz"], dtype=np.float64)
    etov = np.ascontiguousarray(mesh["etov"], dtype=np.int32)
    pid = mesh.get("vertex_periodic_id")
    bc = np.ascontiguousarray(mesh["face_bc"], dtype=np.int8)
    with open(path, "wb") as f:
        f.write(np.int64(vxyz.shape[0]).tobytes())
        f.write(np.int64(etov.shape[0]).tobytes())
        f.write(np.int32(1 if pid is not None else 0).tobytes())
        f.write(vxyz.tobytes())
        f.write(etov.tobytes())
        if pid is not None:
            f.write(np.ascontiguousarray(pid, dtype=np.int32).tobytes())
        f.write(bc.tobytes())


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_host_setup_under_sanitizers(tmp_path):
    exe = str(tmp_path / "driver")
    srcs = [os.path.join(HERE, "host_sanitizer", "driver.cpp")] + [
        os.path.join(CSRC, n) for n in ("refelem.cpp", "mesh.cpp", "order.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-Wno-attributes", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
           "-o", exe] + srcs
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    meshes = {
        "boxed": W.kuhn_cube(3, 1.0),
        "periodic": W.kuhn_cube(3, 1.0, periodic=True),
        "general": W.general_mesh(3, 1.0, seed=7),
        "column": W.kuhn_box(5, 3, 3, 1.25, 0.75, 0.75, periodic=(False, True, True),
                             free_faces=("x+",)),
    }
    files = []
    for name, m in meshes.items():
        p = str(tmp_path / (name + ".bin"))
        _write_mesh(p, m)
        files.append(p)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe] + files, capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "host checks passed" in r.stdout
