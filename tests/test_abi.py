"""The C-ABI library loads, exports every entry point include/mpm.h declares,
and rejects invalid descriptions on the host (no GPU needed)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2503_05046_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mpm():
    from paper_2503_05046_amd import build, mpm as M
    build.build(force=not os.path.exists(M.LIB_PATH))
    M.load()
    return M


def _declared():
    src = open(os.path.join(ROOT, "include", "mpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpm_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(mpm):
    names = _declared()
    assert set(names) == set(mpm.EXPORTED)
    lib = mpm.load()
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_size_and_validation(mpm):
    s = I.plain_cube()
    envs = mpm.env_descs(s)
    d = mpm.make_desc(s, envs)
    n = mpm.mpm_workspace_size(d)
    assert n > 0
    # capacity scales the contact part of the workspace
    d2 = mpm.make_desc(s, envs, max_contacts=100)
    assert mpm.mpm_workspace_size(d2) < n

    def expect_einval(mutate):
        e2 = mpm.env_descs(s)
        dd = mpm.make_desc(s, e2)
        mutate(dd, e2)
        with pytest.raises(mpm.MPMError) as ei:
            mpm.mpm_workspace_size(dd)
        assert ei.value.status == mpm.MPM_EINVAL
        assert mpm.mpm_last_error()

    expect_einval(lambda d, e: setattr(d, "h", 0.0))
    expect_einval(lambda d, e: setattr(d, "N", 0))
    expect_einval(lambda d, e: setattr(d, "struct_size", 8))
    expect_einval(lambda d, e: setattr(d, "max_iter", 0))
    expect_einval(lambda d, e: setattr(e[0], "nu", 0.5))
    expect_einval(lambda d, e: setattr(e[0], "dx", -1.0))
    expect_einval(lambda d, e: setattr(e[0], "eps_s", 0.0))
    expect_einval(lambda d, e: setattr(e[0], "p_end", 10))
    expect_einval(lambda d, e: setattr(e[0], "material", 7))


def test_null_arguments(mpm):
    lib = mpm.load()
    n = ct.c_size_t(0)
    assert lib.mpm_workspace_size(None, ct.byref(n)) == mpm.MPM_EINVAL
    assert lib.mpm_step(None, None, None, None) == mpm.MPM_EINVAL
    lib.mpm_destroy(None)


def test_struct_layouts_match_the_header(mpm, tmp_path):
    """Every ctypes mirror of a struct in include/mpm.h has the header's size
    and field offsets (compiled with the host C compiler; no GPU)."""
    import ctypes as ct
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    pairs = {"EnvDesc": "mpm_env_desc", "Desc": "mpm_desc", "EnvGrad": "mpm_env_grad",
             "RigidGrad": "mpm_rigid_grad", "RigidDesc": "mpm_rigid_desc", "RigidState": "mpm_rigid_state",
             "RigidImpulse": "mpm_rigid_impulse", "StepStats": "mpm_step_stats",
             "ProfileData": "mpm_profile_data"}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpm.h"', "int main(void) {"]
    expect = []
    for py, c in pairs.items():
        cls = getattr(mpm, py)
        lines.append(f'    printf("%zu\\n", sizeof({c}));')
        expect.append((f"sizeof {c}", ct.sizeof(cls)))
        for name, _ in cls._fields_:
            lines.append(f'    printf("%zu\\n", offsetof({c}, {name}));')
            expect.append((f"{c}.{name}", getattr(cls, name).offset))
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    include = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call([cc, "-std=c99", "-I", include, str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert len(got) == len(expect)
    bad = [(what, want, g) for (what, want), g in zip(expect, got) if want != g]
    assert not bad, bad
