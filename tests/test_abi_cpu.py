"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates arguments without a GPU."""
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "lcf.h")).read()
    decl = re.findall(r"^\s*(?:lcf_status|const char\*|int32_t)\s+(lcf_[a-z_0-9]+)\s*\(", txt, re.M)
    return sorted(set(decl))


def test_library_exports_every_declared_symbol(lcf):
    lib = lcf.LIB_PATH
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lcf_[a-z_0-9]+)", out))
    declared = _declared_symbols()
    assert declared, "no declarations parsed"
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(lcf.load(), s)


def test_validate_geometry_and_threshold(lcf):
    thr = lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=4)
    ok = lcf.geometry(64, 64, 32, 3, 3)
    assert lcf.validate(ok, thr) == 0
    assert lcf.validate(lcf.geometry(64, 64, 3, 3, 3), thr) == 1          # nt < 4
    assert lcf.validate(lcf.geometry(64, 64, 32, 65, 3), thr) == 1        # grid > image
    assert lcf.validate(lcf.geometry(64, 64, 32, 2, 2, sigma_frac=0.0), thr) == 1   # flat needs 1x1
    assert lcf.validate(lcf.geometry(64, 64, 32, 1, 1, sigma_frac=0.0), thr) == 0
    assert lcf.validate(lcf.geometry(64, 64, 300, 2, 2), thr) == 2        # nt too large
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_FIXED_K, k_fixed=33)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_KNEE, knee_max_frac=0.0)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_KNEE, beta_knee=-1.0)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=9)) == 1
    assert lcf.validate(ok, lcf.Threshold(pd_mode=3)) == 1
    assert lcf.validate(ok, lcf.Threshold(deflate_rho=-1.0)) == 1
    assert lcf.validate(ok, thr, precision=7) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_MEDIAN, beta_median=1.43)) == 0
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_MEDIAN, beta_median=0.0)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_MEDIAN, beta_median=float("inf"))) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_MEDIAN, shape=lcf.SHAPE_SIGMOID, beta_sigmoid=0.0)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_SLOPE, slope_thr=1.1)) == 0
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_SLOPE, slope_thr=-1.0)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_SLOPE, slope_thr=float("nan"))) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_POWER, beta_power=2.0)) == 0
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_POWER, beta_power=0.0)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_NCC)) == 0
    assert lcf.validate(ok, lcf.Threshold(cut=lcf.CUT_NCC, shape=lcf.SHAPE_SIGMOID, beta_sigmoid=0.0)) == 1
    assert lcf.validate(ok, lcf.Threshold(cut=8)) == 1


def test_abi_version_matches_binding(lcf):
    assert lcf.load().lcf_abi_version() == lcf.ABI_VERSION


def test_python_package_has_no_compute_fallback():
    import paper_2405_11105_amd as m
    src = open(m.__file__).read()
    assert "import oracle" not in src and "from oracle" not in src
    for op in ("linalg", "matmul", "einsum", ".eigh(", " @ ", "fft."):
        assert op not in src, op
