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
