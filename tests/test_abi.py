"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad configurations before touching a device."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbf.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mbf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared()
    for n in ["mbf_create", "mbf_set_material", "mbf_set_pump", "mbf_add_point_source",
              "mbf_set_probes", "mbf_step", "mbf_read_energy", "mbf_read_spectrum",
              "mbf_read_field", "mbf_save_state", "mbf_load_state", "mbf_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_0809_1547_amd import mbf
    out = subprocess.run(["nm", "-D", "--defined-only", mbf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(mbf_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        assert hasattr(mbf.lib, n)


def test_config_defaults():
    from paper_0809_1547_amd import mbf
    c = mbf.mbf_config_default(32, 33, 34)
    assert (c.nx, c.ny, c.nz) == (32, 33, 34)
    assert c.courant == 0.99 and c.dx == 20e-9 and c.lambda0 == 590e-9 and c.dlambda == 230e-9
    assert c.tau21 == 1e-9 and c.Wp == 1e12 and c.noise == 1 and c.precision == mbf.MBF_FP32


@pytest.mark.parametrize("field,value,code", [
    ("courant", 1.01, -2), ("courant", 0.0, -2), ("courant", float("nan"), -2),
    ("nx", 1, -1), ("dx", -1.0, -1), ("tau21", 0.0, -1), ("E_sp", float("inf"), -1),
    ("precision", 7, -1),
])
def test_create_rejects_bad_configs_before_allocating(field, value, code):
    from paper_0809_1547_amd import mbf
    c = mbf.mbf_config_default(8, 8, 8)
    setattr(c, field, value)
    with pytest.raises(mbf.MbfError) as e:
        mbf.mbf_create(c)
    assert e.value.code == code


@pytest.mark.parametrize("n,precision", [((16, 65535, 16), "fp32"), ((16, 16, 70000), "fp32"),
                                         ((1100, 1100, 1100), "fp32"), ((820, 820, 820), "fp64"),
                                         ((1023, 1023, 1023), "fp32")])
def test_create_rejects_grids_beyond_the_limits(n, precision):
    # 16-bit grid rows/planes of the launch and 32-bit site offsets: ny, nz <
    # 65535 and one site array below 4 GiB, checked before any allocation
    # (1023^3 is the first cube past it: 1024^3 sites of 4 bytes; 1023 x 1023
    # x 1022, one plane less, is the largest accepted grid and is stepped in
    # tests/test_gpu_maxsize.py)
    from paper_0809_1547_amd import mbf
    c = mbf.mbf_config_default(*n)
    c.precision = mbf.MBF_FP64 if precision == "fp64" else mbf.MBF_FP32
    with pytest.raises(mbf.MbfError) as e:
        mbf.mbf_create(c)
    assert e.value.code == mbf.MBF_EINVAL


def test_create_bad_boundary():
    from paper_0809_1547_amd import mbf
    c = mbf.mbf_config_default(8, 8, 8)
    c.boundary[1] = 5
    with pytest.raises(mbf.MbfError) as e:
        mbf.mbf_create(c)
    assert e.value.code == mbf.MBF_EINVAL


def test_version_string():
    from paper_0809_1547_amd import mbf
    assert "gfx950" in mbf.mbf_version()
