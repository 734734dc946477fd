"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run on a tiny scene of every SH degree and on the
10k-Gaussian workload-0 camera: any invalid access, leak or undefined
operation fails the run; its render must equal the normal build's."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import scenegen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    out = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "gs_oracle.c"), "-lm", "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-400:])
    return out


def _run(driver, tmp_path, sc, pose, intr, W, H):
    path = str(tmp_path / "case.bin")
    n = len(sc["opacity"])
    with open(path, "wb") as f:
        f.write(np.int64(n).tobytes())
        f.write(np.array([sc["sh_degree"], W, H, 0], np.int32).tobytes())
        for k in ("means", "scales", "quats", "opacity", "sh"):
            f.write(np.ascontiguousarray(sc[k], np.float32).tobytes())
        f.write(np.ascontiguousarray(pose, np.float32).reshape(12).tobytes())
        f.write(np.ascontiguousarray(intr, np.float32).reshape(4).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr, r.stderr[-2000:]
    ref = oracle.render(sc, pose, intr, W, H, bg=(0.1, 0.2, 0.3))
    checksum = float(r.stdout.split("checksum")[1])
    assert checksum == pytest.approx(float(ref.rgb.sum()), rel=1e-9)
    return r.stdout


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_oracle_clean_under_sanitizers_tiny(driver, tmp_path, deg):
    sc = scenegen.tiny_scene(25, 300 + deg, sh_degree=deg, spread=0.7)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    print(_run(driver, tmp_path, sc, pose, np.array([20, 20, 12.3, 9.7]), 24, 18))


def test_oracle_clean_under_sanitizers_workload0(driver, tmp_path):
    sc = scenegen.make_scene(0)
    cams = scenegen.make_cameras(0)
    print(_run(driver, tmp_path, sc, cams["poses"][0], cams["intrinsics"][0], 64, 48))
