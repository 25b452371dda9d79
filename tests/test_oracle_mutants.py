"""The oracle's pins are sharp: each plausible mistake below, planted in a copy of
oracle.cpp (CPU only), makes the pin suite fail.  A mistake no pin catches would be
"parity unpinned"; the list covers each step of the method the oracle computes."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")
# the pins that stand on the paper and the mathematics (closed forms, invariants, brute
# force, the exact definitions); the stored-fixture regression test is left out
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_local.py", "tests/test_oracle_whole.py"]

# (name, the passage whose reading the mistake breaks, text in oracle.cpp, planted text)
MUTANTS = [
    ("gregory-weight-on-pv", "Sec. 2.2 blend, Alg. 2 weighting (reading R1)",
     "double lam = du / den;", "double lam = dv / den;"),
    ("weight-bounds-paired-wrongly", "Sec. 2.2 weight bounds, Alg. 2",
     "double lam_lo = dul / (dul + dvh), lam_hi = duh / (duh + dvl);",
     "double lam_lo = dul / (dul + dvl), lam_hi = duh / (duh + dvh);"),
    ("displacement-dropped", "Sec. 3.2, Alg. 2: d(D)",
     "d = d + (wbar(i, u0, u1) * wbar(j, v0, v1)) * vabs(A - B);", "d = d + 0.0 * vabs(A - B);"),
    ("bernstein-peaks-swapped", "Alg. 2: w-bar peaks at 1/3 and 2/3 (reading R3)",
     "double peak = k == 1 ? 1.0 / 3.0 : 2.0 / 3.0;", "double peak = k == 1 ? 2.0 / 3.0 : 1.0 / 3.0;"),
    ("crop-v-with-u-range", "Alg. 1 / Sec. 2.1 crop to [u0,u1] x [v0,v1]",
     "crop1(in, v0, v1, out);", "crop1(in, u0, u1, out);"),
    ("de-casteljau-wrong-operand", "Sec. 3.1 de Casteljau split",
     "V3 abc = s * ab + t * bc;", "V3 abc = s * ab + t * cd;"),
    ("slab-open-interval", "closed slab test (reading R10)",
     "if (!(near <= far)) return false;", "if (!(near < far)) return false;"),
    ("leaf-uv-at-corner", "reported (u, v) is the leaf centre (reading R9)",
     "best.u = (lpu + csu / 2) * kUnit;", "best.u = lpu * kUnit;"),
    ("farther-child-first", "Sec. 3.3 closest child first",
     "bool first_r = hr && (!hl || tr < tl);", "bool first_r = hr && (!hl || tr > tl);"),
    ("frame-not-orthogonal", "Sec. 3.4 patch-local frame (reading R23)",
     "V3 w = ev - dot(ev, r0) * r0;", "V3 w = ev;"),
    ("frame-boxes-not-grown", "Sec. 3.4 growing boxes to close gaps (reading R23)",
     "Q.pad = std::ldexp(std::max(ext.x, std::max(ext.y, ext.z)), -19);", "Q.pad = 0.0 * ext.x;"),
    ("one-split-short", "fixed leaf depth L per axis (reading R7)",
     "const int leaf_depth = 2 * L;", "const int leaf_depth = 2 * L - 1;"),
]


# Mistakes in the FP64 references of the learned child ordering (oracle/mlp.py: the
# network, its loss and training step; oracle/policy.py: its inputs and labels),
# checked against tests/test_oracle_mlp.py in a copy of the test tree.
PY_MUTANTS = [
    ("relu-gate-dropped", "mlp.py", "backpropagation through the second ReLU",
     'd2 = (d3 @ p["W3"]) * (c["a2"] > 0)', 'd2 = (d3 @ p["W3"])'),
    ("bias-gradient-averaged", "mlp.py", "gradient of the first bias",
     'g["W1"], g["b1"] = d1.T @ c["x"], d1.sum(axis=0)', 'g["W1"], g["b1"] = d1.T @ c["x"], d1.mean(axis=0)'),
    ("bf16-rounds-ties-up", "mlp.py", "bfloat16 rounding to nearest even (reading R22)",
     "b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16", "b = (b + 0x8000) >> 16"),
    ("adam-without-bias-correction", "mlp.py", "Adam's bias-corrected moments",
     "mh = m / (1.0 - beta1 ** t)", "mh = m"),
    ("order-projection-swapped", "mlp.py", "the top grandchild's u-half first (reading R18)",
     "return top >> 1, top & 1", "return top & 1, top >> 1"),
    ("onb-left-handed", "policy.py", "the ray frame of Duff et al. 2017 (reading R17)",
     "e2 = np.array([b, sign + n[1] * n[1] * a, -n[1]])", "e2 = -np.array([b, sign + n[1] * n[1] * a, -n[1]])"),
    ("entry-point-at-exit", "policy.py", "corners relative to the node box's entry point (reading R17)",
     "p = o + min(na, nb) * d", "p = o + max(na, nb) * d"),
    ("label-bits-swapped", "policy.py", "labels name the grandchild holding the leaf (reading R19)",
     "labels[k] = 2 * ((iu >> (L - 1 - k)) & 1) + ((iv >> (L - 1 - k)) & 1)",
     "labels[k] = 2 * ((iv >> (L - 1 - k)) & 1) + ((iu >> (L - 1 - k)) & 1)"),
]


def _run_py(tmp, name, fname, old, new):
    d = os.path.join(tmp, name)
    for sub in ("oracle", "tests", "paper_1811_03510_amd"):
        shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                        ignore=shutil.ignore_patterns("__pycache__", "_build", "*.so", "csrc", "*.o"))
    shutil.copy(os.path.join(ROOT, "oracle", "liboracle.so"), os.path.join(d, "oracle", "liboracle.so"))
    path = os.path.join(d, "oracle", fname)
    text = open(path).read()
    assert text.count(old) == 1, f"{name}: the planted site is no longer in oracle/{fname}"
    with open(path, "w") as f:
        f.write(text.replace(old, new))
    env = {k: v for k, v in os.environ.items() if k != "ORACLE_LIB"}
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_oracle_mlp.py"], cwd=d, env=env, capture_output=True, text=True, timeout=600)
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return name, r.returncode, failed[:1]


def _run(tmp, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"{name}: the planted site is no longer in oracle.cpp"
    d = os.path.join(tmp, name)
    os.makedirs(d, exist_ok=True)
    src, lib = os.path.join(d, "oracle.cpp"), os.path.join(d, "liboracle.so")
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", "-o", lib,
                    src], check=True, capture_output=True)
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return name, r.returncode, failed[:1]


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_every_planted_mistake_fails_a_pin(tmp_path):
    # control: the same harness on an unaltered copy passes, so a failure means the mistake
    site = MUTANTS[0][2]
    with ThreadPoolExecutor(max_workers=4) as ex:
        res = list(ex.map(lambda m: _run(str(tmp_path), m[0], m[2], m[3]), [("control", "", site, site)] + MUTANTS))
    assert res[0][1] == 0, f"the unaltered copy fails the pins: {res[0]}"
    res = res[1:]
    for name, rc, failed in res:
        print(f"{name}: exit {rc} {failed}", flush=True)
    survivors = [name for name, rc, _ in res if rc == 0]
    assert not survivors, f"planted mistakes that no pin catches: {survivors}"


@pytest.mark.slow
def test_every_planted_mistake_in_the_learned_order_references_fails_a_pin(tmp_path):
    assert os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so"))
    site = PY_MUTANTS[0][3]
    with ThreadPoolExecutor(max_workers=4) as ex:
        res = list(ex.map(lambda m: _run_py(str(tmp_path), m[0], m[1], m[3], m[4]),
                          [("control", "mlp.py", "", site, site)] + PY_MUTANTS))
    assert res[0][1] == 0, f"the unaltered copy fails the pins: {res[0]}"
    res = res[1:]
    for name, rc, failed in res:
        print(f"{name}: exit {rc} {failed}", flush=True)
    survivors = [name for name, rc, _ in res if rc == 0]
    assert not survivors, f"planted mistakes that no pin catches: {survivors}"
