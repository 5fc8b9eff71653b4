"""The oracle's pins catch plausible mistakes: each case plants one mistake in
a copy of the oracle's C source (on the CPU), builds it, and runs the pin
suites against it; at least one pin must fail."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_rng.py", "tests/test_oracle_math.py", "tests/test_oracle_pso.py"]

MUTATIONS = {
    "cognitive_sign": ("((pr->c1 * r[0]) * (pi - xi))", "((pr->c1 * r[0]) * (xi - pi))"),
    "social_operand": ("((pr->c2 * r[1]) * (g[d] - xi))", "((pr->c2 * r[1]) * (xi - g[d]))"),
    "social_dropped": (" + ((pr->c2 * r[1]) * (g[d] - xi));", ";"),
    "r1_reused": ("(pr->c2 * r[1])", "(pr->c2 * r[0])"),
    "inertia_on_position": ("(pr->w * vi)", "(pr->w * xi)"),
    "philox_lane": ("out[0] = oracle_uniform_f32(r[2 * (d & 1)]);", "out[0] = oracle_uniform_f32(r[(2 * (d & 1)) ^ 2]);"),
    "philox_weyl": ("k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;"),
    "philox_rounds": ("round < 10; ++round", "round < 9; ++round"),
    "uniform_bits": ("(float)(u >> 8) * 0x1p-24f", "(float)(u >> 9) * 0x1p-24f"),
    "pbest_non_strict": ("if (f < pf[i]) {\n        pf[i] = f;\n        for (int d = 0; d < D; ++d) p[d * N + i] = x[d * N + i];\n    }\n}",
                         "if (f <= pf[i]) {\n        pf[i] = f;\n        for (int d = 0; d < D; ++d) p[d * N + i] = x[d * N + i];\n    }\n}"),
    "tie_highest_index": ("<< 32) | i; }", "<< 32) | (0xFFFFFFFFu - i); }"),
    "rastrigin_sign": ("acc = acc + (z * z - 10.0f *", "acc = acc + (z * z + 10.0f *"),
    "rosenbrock_index": ("float a = zn - zd * zd;", "float a = zd - zn * zn;"),
    "ackley_coeff": ("-0.2f * sqrtf(m1)", "-0.25f * sqrtf(m1)"),
    "cubic_coeff": ("- 0.8f * z2)", "- 0.9f * z2)"),
    "cos_coeff": ("0x1.03c1f0p+2f", "0x1.03c1e0p+2f"),
    "exp_reduction": ("r = fmaf(-k, LN2_LO, r);", "r = r;"),
    "no_position_clamp": ("float xn = clampf(xi + vn, pr->lo, pr->hi);", "float xn = xi + vn;"),
    "no_velocity_clamp": ("vn = clampf(vn, -pr->vmax, pr->vmax);\n        /* Eq. 2", "/* Eq. 2"),
    "fitness_of_old_position": ("        x[e] = xn;\n        v[e] = vn;\n    }\n    /* Step 3",
                                "        v[e] = vn;\n        p[e] = p[e] + 0.0f * xn;\n    }\n    /* Step 3"),
    "gbest_not_refreshed": ("    *gkey = k;\n    gather_f32(pr, p, k, gpos);\n    return 1;", "    *gkey = k;\n    return 1;"),
    "init_same_draw": ("pr->lo + span * u[0]", "pr->lo + span * u[1]"),
    "stop_off_by_one": ("if (tol > 0.0f && fabsf(key_value_f32(gkey) - f_star) < tol) break;\n        ++t;",
                        "++t;\n        if (tol > 0.0f && fabsf(key_value_f32(gkey) - f_star) < tol) break;"),
}


@pytest.fixture(scope="module")
def kat_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        return None
    from tests.test_oracle_rng import ROCRAND_PROG
    d = tmp_path_factory.mktemp("kat")
    (d / "kat.cpp").write_text(ROCRAND_PROG)
    subprocess.run([hipcc, "-O1", str(d / "kat.cpp"), "-o", str(d / "kat")], check=True, capture_output=True)
    return str(d / "kat")


def _run_pins(name, lib, kat):
    env = dict(os.environ, PSO_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    if kat:
        env["PSO_ROCRAND_KAT_EXE"] = kat
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_FILES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-400:]


def test_every_planted_mistake_fails_a_pin(tmp_path, kat_exe):
    src = open(oracle.oracle.SRC).read()
    jobs = []
    for name, (old, new) in MUTATIONS.items():
        assert src.count(old) >= 1, f"mutation {name} does not apply"
        msrc = tmp_path / f"{name}.c"
        msrc.write_text(src.replace(old, new, 1))
        lib = str(tmp_path / f"lib_{name}.so")
        oracle.oracle.build(out=lib, src=str(msrc))
        jobs.append((name, lib))
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda j: _run_pins(j[0], j[1], kat_exe), jobs))
    survived = [(n, out) for n, rc, out in results if rc == 0]
    assert not survived, f"mistakes no pin caught: {[n for n, _ in survived]}"


def test_unmutated_oracle_passes_pins(kat_exe):
    name, rc, out = _run_pins("none", oracle.oracle.LIB, kat_exe)
    assert rc == 0, out
