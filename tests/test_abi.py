"""The C ABI library loads, exports every declared symbol and validates its arguments before
touching a GPU (runs without one)."""
import ctypes
import os
import re

import pytest

from paper_2404_18034_amd import api
from paper_2404_18034_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "scp_batch.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(scp_batch_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(api.LIB_PATH):
        pytest.skip("libscp_batch.so not built")
    return api.load()


def test_exports_match_header(lib):
    decl = declared_functions()
    assert decl == sorted(api.EXPORTS)
    for name in decl:
        assert hasattr(lib, name), name


def test_workspace_bytes_and_validation(lib):
    cfg = I.solver_settings("C1")
    s = api.make_settings(cfg, "f32", 20, 1024)
    n1 = api.workspace_bytes(s)
    s2 = api.make_settings(cfg, "f32", 20, 2048)
    s3 = api.make_settings(cfg, "f64", 20, 1024)
    assert n1 > 0 and api.workspace_bytes(s2) > n1 and api.workspace_bytes(s3) > n1
    assert n1 % 256 == 0
    for bad in (dict(k_max=1), dict(k_max=51), dict(w_prox=0.0), dict(rho=2.0),
                dict(pipg_iters_max=0), dict(dtype=7), dict(power_fp32=2), dict(power_fp32=-1)):
        sb = api.make_settings(cfg, "f32", 20, 1024)
        for k, v in bad.items():
            setattr(sb, k, v)
        assert api.workspace_bytes(sb) == 0
    # node projections need block-uniform scales (the paper's set alone does not)
    px = (1, 4, 4, 3, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 0.1)
    sb = api.make_settings(dict(cfg, px=px, node_projections=31), "f32", 20, 1024)
    assert api.workspace_bytes(sb) == 0
    sb = api.make_settings(dict(cfg, px=px, node_projections=0), "f32", 20, 1024)
    assert api.workspace_bytes(sb) == n1
    # the power-iteration precision setting needs no extra workspace
    assert api.workspace_bytes(api.make_settings(dict(cfg, power_fp32=1), "f32", 20, 1024)) == n1


def test_create_rejects_bad_workspace_before_any_hip_call(lib):
    cfg = I.solver_settings("C1")
    s = api.make_settings(cfg, "f32", 20, 16)
    h = ctypes.c_void_p()
    rc = lib.scp_batch_create(ctypes.byref(s), 0, None, None, 0, ctypes.byref(h))
    assert rc == 6 and not h.value
    assert b"workspace" in lib.scp_batch_create_error()
    rc = lib.scp_batch_create(ctypes.byref(s), 0, None, ctypes.c_void_p(256 + 8),
                              ctypes.c_size_t(1 << 30), ctypes.byref(h))
    assert rc == 6 and b"aligned" in lib.scp_batch_create_error()
    s.k_max = 0
    rc = lib.scp_batch_create(ctypes.byref(s), 0, None, None, 0, ctypes.byref(h))
    assert rc == 1


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.scp_batch_solve(None, None, None) == 1
    assert lib.scp_batch_set_stream(None, None) == 1
    assert lib.scp_batch_destroy(None) == 1
    assert lib.scp_batch_last_error(None) == b"null handle"


def test_struct_layouts_match_the_header(tmp_path):
    # the ctypes mirrors and the C declarations agree on every field offset and size
    structs = {"scp_settings": api.Settings, "scp_problem": api.Problem,
               "scp_solution": api.Solution, "scp_lastiter": api.LastIter}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "scp_batch.h"',
             'int main(void) {']
    for cname, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append('return 0; }')
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(cls, f).offset, (cname, f)


def test_gradient_settings_validated(lib):
    cfg = I.solver_settings("C3")
    s = api.make_settings(cfg, "f32", 20, 64)
    n_grad = api.workspace_bytes(s)
    s0 = api.make_settings(dict(cfg, grad_pipg_steps=0), "f32", 20, 64)
    assert 0 < api.workspace_bytes(s0) < n_grad
    bad = api.make_settings(dict(cfg, grad_ckpt_every=0), "f32", 20, 64)
    assert api.workspace_bytes(bad) == 0
    bad = api.make_settings(dict(cfg, grad_ckpt_every=201), "f32", 20, 64)
    assert api.workspace_bytes(bad) == 0


def test_scalar_dilation_setting_validated(lib):
    # 0 and 1 are accepted (same workspace: the variant needs no device memory of its own),
    # other values are rejected; the combinations it does not implement are refused at
    # create time (a GPU test covers that)
    cfg = I.solver_settings("C1")
    n0 = api.workspace_bytes(api.make_settings(dict(cfg, scalar_dilation=0), "f32", 20, 64))
    n1 = api.workspace_bytes(api.make_settings(dict(cfg, scalar_dilation=1), "f32", 20, 64))
    assert n0 > 0 and n1 == n0
    for v in (2, -1):
        assert api.workspace_bytes(api.make_settings(dict(cfg, scalar_dilation=v),
                                                     "f32", 20, 64)) == 0


def test_tuning_variant_count_matches_header():
    import re
    from paper_2404_18034_amd import api
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "scp_batch.h")).read()
    n = int(re.search(r"#define SCP_TUNE_VARIANTS (\d+)", hdr).group(1))
    assert n == len(api.TUNE_VARIANTS)
    k = int(re.search(r"#define SCP_KERNEL_CLASSES (\d+)", hdr).group(1))
    assert k == len(api.KERNEL_CLASSES)
