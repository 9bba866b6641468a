"""Host-side checks of the C interface (no GPU needed): the library loads, exports every entry
point declared in include/wfq.h, and rejects bad arguments before touching a device."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2103_00438_amd", "libwfq.so")


def declared_functions():
    with open(os.path.join(ROOT, "include", "wfq.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wfq_[a-z_A-Z]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("wfq_build", "wfq_solve", "wfq_solve_dev", "wfq_serve", "wfq_submit", "wfq_poll",
                     "wfq_wait", "wfq_serve_stats", "wfq_serve_stop", "wfq_destroy", "wfq_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build libwfq.so first (python -m paper_2103_00438_amd.build)"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2103_00438_amd import wfq
    for name in declared_functions():
        assert name in wfq._SIGNATURES, name
        assert hasattr(wfq, name), name


def test_argument_errors_before_device():
    from paper_2103_00438_amd import wfq
    import wfq_inputs as wi
    p = dict(wi.workloads.GRAPHENE)
    with pytest.raises(wfq.WfqError) as e:
        wfq.wfq_build(np.zeros((1, 3)), p)           # N < 2
    assert e.value.code == wfq.WFQ_EINVAL
    bad = np.zeros((3, 3))
    bad[1, 0] = np.nan
    with pytest.raises(wfq.WfqError) as e:
        wfq.wfq_build(bad, p)
    assert e.value.code == wfq.WFQ_EINVAL
    with pytest.raises(wfq.WfqError) as e:
        wfq.wfq_build(np.eye(3), dict(p, eta=-1.0))
    assert e.value.code == wfq.WFQ_EINVAL
    with pytest.raises(wfq.WfqError) as e:
        wfq.wfq_build(np.eye(3), dict(p, cutoff_eps=0.7))
    assert e.value.code == wfq.WFQ_EINVAL
    assert "cutoff_eps" in wfq.wfq_last_error()


def test_null_handle_is_rejected():
    from paper_2103_00438_amd import wfq
    lib = wfq.load()
    assert lib.wfq_info(None, None, None, None) == wfq.WFQ_EINVAL
    lib.wfq_destroy(None)
    lib.wfq_serve_stop(None)


def test_block_product_variant_registry():
    # every precision has the narrow kernels and the 128 x 256 tile; FP32 and BF16 add the wide
    # column tiles (their accumulators are half the size of FP64 ones)
    from paper_2103_00438_amd import wfq
    names = {p: [n for n, _ in wfq.wfq_tx_variants(p)] for p in ("fp64", "fp32", "bf16")}
    for p, v in names.items():
        assert len(v) == len(set(v))
        assert {"skinny2", "skinny4", "skinny8", "m128n256w8", "m32n128"} <= set(v)
    wide = {"m96n256w8", "m160n256w8", "m192n256w8", "m192n128w8"}
    assert wide <= set(names["fp32"]) and wide <= set(names["bf16"])
    assert not wide & set(names["fp64"])


def test_binding_structs_match_the_header_layout(tmp_path):
    # the ctypes mirrors of the header's structs: same size and the same offset for every field
    # (a field added on one side only would shift every later one), measured by a C probe
    import shutil
    import subprocess
    from paper_2103_00438_amd import wfq
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = {"wfq_geometry": wfq.Geometry, "wfq_params": wfq.Params, "wfq_solve_opts": wfq.SolveOpts,
             "wfq_result": wfq.Result, "wfq_serve_cfg": wfq.ServeCfg, "wfq_job": wfq.Job,
             "wfq_job_timing": wfq.JobTiming, "wfq_stats": wfq.Stats, "wfq_species": wfq.Species}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "wfq.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_material_closure_of_the_library_equals_the_oracle():
    # the library computes W = 2 n0 A from the material data by the same sum-rule closure as the
    # oracle (host code of libwfq; no device needed): graphene at two Fermi energies, the FCC metal
    # with one and with two free electrons per atom and m* = 1 or 1.5
    from paper_2103_00438_amd import wfq
    from oracle import wfq_oracle as O
    import wfq_inputs as wi
    for base, extra in ((wi.workloads.GRAPHENE, dict(fermi_energy_eV=0.4)),
                        (wi.workloads.GRAPHENE, dict(fermi_energy_eV=1.51)),
                        (wi.workloads.FCC_METAL, dict(valence=1.0, eff_mass=1.0)),
                        (wi.workloads.FCC_METAL, dict(valence=2.0, eff_mass=1.5))):
        p = dict(base, **extra)
        p.pop("W", None)
        assert wfq.wfq_material_weight(p) == pytest.approx(O.material_weight(p), rel=1e-12)
    assert wfq.wfq_material_weight(dict(wi.workloads.GRAPHENE, W=0.05)) == 0.05   # the override
    with pytest.raises(wfq.WfqError) as e:
        wfq.wfq_material_weight(dict(wi.workloads.GRAPHENE, material=None, W=0.0))
    assert e.value.code == wfq.WFQ_EINVAL


def test_isotropic_sigma_helper():
    # Eq. (iso-cross) on the host: the mean of the three sigma_k for orthonormal directions, and a
    # clear error for directions that are not
    from paper_2103_00438_amd import wfq
    lib = wfq.load()
    c, s = math.cos(0.3), math.sin(0.3)
    dirs = np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]])
    info = (wfq.Result * 6)()
    vals = [1.0, 2.0, 6.0, 0.5, 0.25, 0.0]
    for i, v in enumerate(vals):
        info[i].sigma = v
    iso = np.zeros(2)
    assert lib.wfq_isotropic_sigma(wfq._dp(dirs), info, 2, wfq._dp(iso)) == wfq.WFQ_OK
    assert iso[0] == pytest.approx(3.0) and iso[1] == pytest.approx(0.25)
    bad = dirs.copy()
    bad[2] = [0.0, 0.6, 0.8]
    assert lib.wfq_isotropic_sigma(wfq._dp(bad), info, 2, wfq._dp(iso)) == wfq.WFQ_EINVAL
