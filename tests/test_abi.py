"""The C ABI library loads and exports every entry point include/mts.h declares; host-side
parameter validation rejects bad input before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mts.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mts_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2507_11172_amd import mts
    return mts.load_library()


def test_every_declared_symbol_is_exported(lib):
    from paper_2507_11172_amd import mts
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mts.EXPORTS)


def test_status_strings(lib):
    assert lib.mts_status_string(0) == b"MTS_OK"
    assert lib.mts_status_string(-3) == b"MTS_ERR_NOT_MULTIPLE_OF_K"


def _init(lib, **over):
    from paper_2507_11172_amd import mts
    kw = dict(epsilon=1.0, sigma=1.0, rc_pair=2.5, nu=0.073, rc_triplet=2.5, mass=1.0, dt=0.001,
              skin=0.0, k=10, precision=0, lj_energy_shift=1, method=0)
    n = over.pop("n", [500])
    box = over.pop("box", [[8.55, 8.55, 8.55]])
    kw.update(over)
    p = mts.mts_params(**kw)
    nn = np.ascontiguousarray(np.asarray(n, dtype=np.int64))
    bb = np.ascontiguousarray(np.asarray(box, dtype=np.float64))
    h = C.c_void_p()
    rc = lib.mts_init_system(C.byref(p), len(n), nn.ctypes.data_as(C.POINTER(C.c_int64)),
                             bb.ctypes.data_as(C.POINTER(C.c_double)), None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("bad,code", [
    (dict(k=0), -1), (dict(dt=0.0), -1), (dict(mass=-1.0), -1), (dict(sigma=0.0), -1),
    (dict(rc_pair=float("nan")), -1), (dict(precision=7), -1), (dict(method=2), -1),
    (dict(epsilon=-1.0), -1), (dict(skin=-0.1), -1), (dict(skin=float("inf")), -1),
    (dict(n=[-5]), -1),
    (dict(box=[[4.9, 8.5, 8.5]]), -2), (dict(box=[[8.5, 8.5, 5.0]]), -2),
    (dict(rc_triplet=4.3), -2),
    (dict(k_outer=-1), -1), (dict(k_outer=2), -1), (dict(k_outer=2, rc_triplet_inner=2.5), -1),
    (dict(k_outer=2, rc_triplet_inner=-1.0), -1), (dict(k_outer=1, rc_triplet_inner=2.0), -1),
    (dict(k_outer=2, rc_triplet_inner=float("nan")), -1),
    (dict(k_outer=3, rc_triplet_inner=2.0, method=1), -8),
])
def test_host_validation(lib, bad, code):
    rc, h = _init(lib, **bad)
    assert rc == code
    assert not h.value


def test_null_arguments(lib):
    assert lib.mts_init_system(None, 1, None, None, None, None) == -1
    assert lib.mts_sync(None) == -1
    assert lib.mts_respa_step(None, None, None, 0, None) == -1
    assert lib.mts_autotune(None, None, None, 0, None) == -1
    assert lib.mts_get_tuning(None, None) == -1
    assert lib.mts_set_option(None, 1, 1) == -1
    lib.mts_destroy_system(None)  # ignored


def test_params_struct_matches_header(lib):
    """The binding's mts_params mirrors the header's field order and types."""
    import re
    from paper_2507_11172_amd import mts
    hdr = open(os.path.join(ROOT, "include", "mts.h")).read()
    start = hdr.index("typedef struct {", hdr.index("Interaction and integration parameters"))
    body = hdr[start:hdr.index("} mts_params;")]
    fields = re.findall(r"^\s*(double|int32_t)\s+(\w+);", body, re.M)
    py = [(n, t) for n, t in mts.mts_params._fields_]
    assert [f[1] for f in fields] == [n for n, _ in py]
    for (ctype, _), (_, t) in zip(fields, py):
        assert (ctype == "double") == (t is C.c_double)


def test_tuning_struct_matches_header(lib):
    """The binding's mts_tuning mirrors the header's field order and types."""
    import re
    from paper_2507_11172_amd import mts
    hdr = open(os.path.join(ROOT, "include", "mts.h")).read()
    body = hdr[hdr.index("typedef struct {", hdr.index("---- autotuning")):hdr.index("} mts_tuning;")]
    fields = re.findall(r"^\s*(double|int32_t)\s+(\w+);", body, re.M)
    py = [(n, t) for n, t in mts.mts_tuning._fields_]
    assert [f[1] for f in fields] == [n for n, _ in py]
    for (ctype, _), (_, t) in zip(fields, py):
        assert (ctype == "double") == (t is C.c_double)



def test_enum_constants_match_header():
    """Every MTS_ constant the binding defines has the header's value."""
    from paper_2507_11172_amd import mts
    hdr = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "mts.h")).read(), flags=re.S)
    values = {n: int(v) for n, v in re.findall(r"\b(MTS_[A-Z0-9_]+)\s*=\s*(-?\d+)", hdr)}
    ours = {n: getattr(mts, n) for n in dir(mts) if n.startswith("MTS_OPT_")}
    assert ours and set(ours) <= set(values)
    for n, v in ours.items():
        assert values[n] == v, n
    assert values["MTS_OPT_LIST_LANES"] == 2

def test_algorithm1_parameters():
    """Algorithm 1's full step delta_t of P sub-steps maps to dt = delta_t / P, k = P; a
    nested handle's full step spans k * k_outer inner steps."""
    from paper_2507_11172_amd import mts
    p = mts.Params.algorithm1(0.004, 4, nu=0.3)
    assert p.dt == 0.004 / 4 and p.k == 4 and p.nu == 0.3 and p.span == 4
    assert mts.Params(k=2, k_outer=5, rc_triplet_inner=2.0).span == 10
    with pytest.raises(ValueError):
        mts.Params.algorithm1(0.004, 0)


C_PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "mts.h"
int main(void) {
    mts_params p;
    memset(&p, 0, sizeof p);
    p.epsilon = 1.0; p.sigma = 1.0; p.rc_pair = 2.5; p.nu = 0.073; p.rc_triplet = 2.5;
    p.mass = 1.0; p.dt = 0.001; p.k = 0;  /* invalid: k < 1 */
    int64_t n = 10;
    double box[3] = {10.0, 10.0, 10.0};
    mts_system *s = (mts_system *)&p;
    mts_status r = mts_init_system(&p, 1, &n, box, NULL, &s);
    printf("%s %s\n", mts_status_string(r), mts_status_string(MTS_ERR_NOT_MULTIPLE_OF_K));
    return (r == MTS_ERR_INVALID_ARG && s == NULL) ? 0 : 1;
}
"""


def test_header_is_c99_and_library_links_from_c(lib, tmp_path):
    """The boundary is a C ABI: the header compiles as strict C99 without warnings, and a
    plain C program linked against libmts.so gets host-side validation through it."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "abi"
    libdir = os.path.join(ROOT, "paper_2507_11172_amd")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"), str(src), "-L", libdir, "-lmts",
                    "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.split() == ["MTS_ERR_INVALID_ARG", "MTS_ERR_NOT_MULTIPLE_OF_K"]
