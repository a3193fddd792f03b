"""The C-ABI from C: include/lbm.h compiles as strict C99, a C client links liblbm.so and runs the
host-only calls (no GPU), and the struct layouts it sees are the ones the Python binding uses.
A field added to a struct on one side only shows up here as a size or offset mismatch."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2007_12266_amd import inputs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = os.path.join(ROOT, "tests", "capi", "abi_probe.c")


@pytest.fixture(scope="module")
def probe_output(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    lib = lbm.load_library()._name
    out = str(tmp_path_factory.mktemp("capi") / "abi_probe")
    libdir = os.path.dirname(os.path.abspath(lib))
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(ROOT, "include"), PROBE, "-o", out,
                    "-L", libdir, "-l:" + os.path.basename(lib), "-Wl,-rpath," + libdir],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([out], check=True, capture_output=True, text=True, timeout=120)
    rows = {}
    for line in r.stdout.splitlines():
        key, _, rest = line.partition(" ")
        rows[key] = rest.split()
    return rows


def test_struct_layouts_match_the_binding(probe_output):
    sizes = {"lbm_params": lbm.Params, "lbm_tuning": lbm.Tuning, "lbm_domain_info": lbm.Info,
             "lbm_reduction": lbm.Reduction, "lbm_timing": lbm.Timing}
    for cname, py in sizes.items():
        assert int(probe_output["sizeof." + cname][0]) == ctypes.sizeof(py), cname
    fields = {"lbm_params": lbm.Params, "lbm_tuning": lbm.Tuning, "lbm_domain_info": lbm.Info,
              "lbm_reduction": lbm.Reduction, "lbm_timing": lbm.Timing}
    for key, val in probe_output.items():
        struct, _, field = key.partition(".")
        if struct in fields:
            assert int(val[0]) == getattr(fields[struct], field).offset, key


def test_host_calls_from_c_agree_with_the_binding(probe_output):
    nx, ny, nz = 7, 6, 5
    labels = np.where(np.arange(nx * ny * nz) % 3 == 0, 0, 1).astype(np.int32)
    prob = inputs.Problem(labels=labels.reshape(nz, ny, nx),
                          label_kind=np.array([inputs.KIND_SOLID, inputs.KIND_FLUID_A], np.int8),
                          label_affinity=np.array([0.25, 0.0]), periodic=(True, True, True),
                          tau_a=1.0, tau_b=1.0, alpha=0.005, beta=0.95)
    q = lbm.prepass_query(prob)
    status, n_pore, n_tail = (int(x) for x in probe_output["prepass_query"])
    assert status == lbm.LBM_OK
    assert (n_pore, n_tail) == (q["n_pore"], len(q["tail_phi"]))
    st, table = (int(x) for x in probe_output["footprint_table"])
    assert st == lbm.LBM_OK and table == lbm.footprint(prob, lbm.FP64,
                                                       neighbour_mode=lbm.NBR_TABLE)
    st, auto = (int(x) for x in probe_output["footprint_auto"])
    assert st == lbm.LBM_OK and auto == lbm.footprint(prob, lbm.FP64)
    st, has_msg = (int(x) for x in probe_output["bad_tau"])
    assert st == lbm.LBM_ERR_ARG and has_msg == 1
    assert probe_output["version"]
