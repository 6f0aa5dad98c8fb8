"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, and the oracle's determinism.

The FP64 oracle, the C ABI's host layer (argument validation, workspace sizing, the BVH
builder, the timing hooks) and the host BVH builder are compiled with g++
-fsanitize=address,undefined -fno-sanitize-recover=all and exercised in child processes with
the sanitizer runtime preloaded; any finding aborts the child. The HIP objects linked beside
the sanitized ABI layer are the regular ones (device code is not instrumented). The sanitized
oracle's outputs must equal the regular build's bit for bit, and two runs of the oracle with
different thread counts must too (its per-pixel work does not depend on scheduling)."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle as O
from paper_2608_24109_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2608_24109_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_2608_24109_amd", "_build")
SAN = ["-O1", "-g", "-std=c++17", "-fPIC", "-pthread", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
HIP_INC = ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"


@pytest.fixture(scope="module")
def san(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    libs = {}
    libs["oracle"] = str(d / "liboracle_san.so")
    _run(["g++", *SAN, "-fopenmp", "-ffp-contract=off", "-shared", "-o", libs["oracle"],
          os.path.join(ROOT, "oracle", "oracle.cpp")])
    libs["bvh"] = str(d / "bvh_check_san.so")
    _run(["g++", *SAN, *HIP_INC, "-shared", "-o", libs["bvh"], os.path.join(HERE, "bvh_check.cpp"),
          os.path.join(CSRC, "bvh_build.cpp")])
    hip_objs = sorted(os.path.join(OBJ, f) for f in os.listdir(OBJ) if f.endswith(".hip.o")) if os.path.isdir(OBJ) else []
    if not hip_objs:
        from paper_2608_24109_amd import build as B
        B.build()
        hip_objs = sorted(os.path.join(OBJ, f) for f in os.listdir(OBJ) if f.endswith(".hip.o"))
    host = []
    for s in ("abi.cpp", "bvh_build.cpp", "timing.cpp"):
        o = str(d / (s + ".o"))
        _run(["g++", *SAN, *HIP_INC, "-c", os.path.join(CSRC, s), "-o", o])
        host.append(o)
    libs["abi"] = str(d / "libexm_san.so")
    _run(["g++", "-shared", "-pthread", "-fsanitize=address,undefined", "-o", libs["abi"], *host, *hip_objs,
          "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    libs["dir"] = str(d)
    return libs


def _child(*args):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, os.path.join(HERE, "sanitized_checks.py"), *args], capture_output=True,
                       text=True, env=env, cwd=ROOT, timeout=900)
    assert r.returncode == 0, f"sanitized child failed ({r.returncode}):\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r.stdout


def test_abi_host_layer_under_sanitizers(san):
    out = _child("abi", san["abi"])
    assert "validation tests passed" in out


def test_bvh_builder_under_sanitizers(san):
    out = _child("bvh", san["bvh"])
    assert "invariants hold" in out


def test_oracle_under_sanitizers_equals_regular_build(san):
    path = os.path.join(san["dir"], "oracle_san.npz")
    _child("oracle", san["oracle"], path)
    import sanitized_checks as S
    ref = S.oracle_outputs(O, I)
    got = np.load(path)
    assert sorted(got.files) == sorted(ref)
    for k in ref:
        assert np.array_equal(np.asarray(ref[k]), got[k], equal_nan=True), k


def test_oracle_is_deterministic():
    """Two renders of the same pixels, on 1 and on 8 threads, agree bit for bit (every output,
    the forward-mode derivative included)."""
    pos, tri = I.interlocking_tori(32, 12)
    cams = I.ring_cameras(1, 4.5, 48, 48)
    sc = I.make_scene("tori_det", pos, tri, 64, 64, 16, 32, 1.0, cams, N_d=8, N_b=2, N_s=2)
    om = O.OracleMesh(sc.pos, sc.tri, sc.uv, sc.tri_uv)
    tab = O.EnvTables(sc.env)
    u = np.random.default_rng(3).normal(size=sc.env.shape)
    runs = [O.render(om, cams[0], tab, sc.tex, sc.env, N_d=8, N_b=2, N_s=2, seed=sc.seed, tmin=sc.tmin,
                     env_dot=u, n_threads=nt) for nt in (1, 8)]
    for k in runs[0]:
        assert np.array_equal(runs[0][k], runs[1][k]), k
    assert np.abs(runs[0].L_ind).max() > 0 and np.abs(runs[0].dL_dir).max() > 0
