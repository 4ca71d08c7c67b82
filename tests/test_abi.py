"""CPU checks of the C ABI boundary: the library loads, exports every entry
point include/amrvac.h declares, and rejects invalid block lists on the host
(no device needed)."""
import os
import re

import numpy as np
import pytest

from conftest import ROOT
from paper_1407_2052_amd import amrvac as A

HEADER = os.path.join(ROOT, "include", "amrvac.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(amrvac_[a-z_]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    assert declared_functions() == sorted(A.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = A.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_abi_version_matches_header():
    m = re.search(r"#define AMRVAC_ABI_VERSION (\d+)", open(HEADER).read())
    assert A.lib().amrvac_abi_version() == int(m.group(1)) == A.ABI_VERSION


def test_header_constants_match_binding():
    src = open(HEADER).read()
    assert re.search(r"#define AMRVAC_NGHOST (\d+)", src).group(1) == str(A.NGHOST)
    for name, val in [("AMRVAC_ERR_INVALID", A.ERR_INVALID), ("AMRVAC_ERR_NONPHYSICAL", A.ERR_NONPHYSICAL),
                      ("AMRVAC_ERR_UNSUPPORTED", A.ERR_UNSUPPORTED), ("AMRVAC_SSPRK54", A.SSPRK54),
                      ("AMRVAC_EXEC_BATCHED", A.EXEC_BATCHED), ("AMRVAC_MHD", A.MHD),
                      ("AMRVAC_MP5", A.MP5), ("AMRVAC_LIM03", A.LIM03), ("AMRVAC_GLM", A.GLM)]:
        assert re.search(rf"{name} = (\d+)", src).group(1) == str(val)


def test_create_rejects_invalid_config_without_device():
    import ctypes
    L = A.lib()
    h = ctypes.c_void_p()
    assert L.amrvac_create(None, None, ctypes.byref(h)) == A.ERR_INVALID
    for cfg in (A.Config(0, A.HD, 1.4, A.EXEC_BATCHED), A.Config(4, A.HD, 1.4, A.EXEC_BATCHED),
                A.Config(2, 7, 1.4, A.EXEC_BATCHED), A.Config(2, A.HD, 1.0, A.EXEC_BATCHED),
                A.Config(2, A.HD, float("nan"), A.EXEC_BATCHED), A.Config(2, A.HD, 1.4, 9),
                A.Config(2, A.HD, 1.4, A.EXEC_BATCHED, 2), A.Config(2, A.HD, 1.4, A.EXEC_BATCHED, -1),
                A.Config(2, 3, 1.4, A.EXEC_BATCHED), A.Config(2, A.HD, 1.4, A.EXEC_BATCHED, 0, 0.1),
                A.Config(2, A.GLM, 1.4, A.EXEC_BATCHED, 0, 0.1), A.Config(2, A.MHD, 1.4, A.EXEC_BATCHED, 0, -1.0),
                A.Config(2, A.MHD, 1.4, A.EXEC_BATCHED, 0, float("inf"))):
        assert L.amrvac_create(ctypes.byref(cfg), None, ctypes.byref(h)) == A.ERR_INVALID
        assert h.value is None
    assert b"invalid config" in L.amrvac_last_error(None)


def grid2(nbx=2, nby=2, n=16):
    nb = nbx * nby
    ns = [[n, n, 1]] * nb
    dx = [[0.1, 0.1, 1.0]] * nb
    xlo = [[0.0, 0.0, 0.0]] * nb
    nbr = []
    for b in range(nb):
        x, y = b % nbx, b // nbx
        nbr.append([y * nbx + (x - 1) % nbx, y * nbx + (x + 1) % nbx,
                    ((y - 1) % nby) * nbx + x, ((y + 1) % nby) * nbx + x, -1, -1])
    return [1000 + b for b in range(nb)], ns, dx, xlo, nbr


def test_validate_accepts_a_periodic_grid():
    st, msg = A.validate_blocks(2, True, 5 / 3, *grid2())
    assert st == A.OK, msg


@pytest.mark.parametrize("mutate,expect", [
    (lambda p, n, dx, x, nb: p.__setitem__(0, 0), "u is NULL"),
    (lambda p, n, dx, x, nb: n.__setitem__(0, [2, 16, 1]), "< 3"),
    (lambda p, n, dx, x, nb: n.__setitem__(0, [16, 16, 2]), "must be 1"),
    (lambda p, n, dx, x, nb: dx.__setitem__(1, [0.0, 0.1, 1.0]), "dx"),
    (lambda p, n, dx, x, nb: dx.__setitem__(1, [float("inf"), 0.1, 1.0]), "dx"),
    (lambda p, n, dx, x, nb: nb.__setitem__(0, [7, 1, 2, 2, -1, -1]), "out of range"),
    (lambda p, n, dx, x, nb: nb.__setitem__(0, [1, 1, 2, 2, 0, -1]), "inactive"),
    (lambda p, n, dx, x, nb: nb.__setitem__(0, [1, 1, 3, 2, -1, -1]), "point back"),
    (lambda p, n, dx, x, nb: n.__setitem__(1, [16, 8, 1]), "face size"),
])
def test_validate_rejects(mutate, expect):
    p, n, dx, x, nb = grid2()
    n = [list(r) for r in n]; dx = [list(r) for r in dx]; nb = [list(r) for r in nb]
    mutate(p, n, dx, x, nb)
    st, msg = A.validate_blocks(2, True, 5 / 3, p, n, dx, x, nb)
    assert st == A.ERR_INVALID
    assert expect in msg, msg


def test_validate_rejects_empty_and_bad_config():
    st, msg = A.validate_blocks(2, True, 5 / 3, [], [], [], [], [])
    assert st == A.ERR_INVALID
    st, msg = A.validate_blocks(2, True, 0.5, *grid2())
    assert st == A.ERR_INVALID and "config" in msg


def test_fixed_faces_need_no_neighbour():
    p, n, dx, x, nb = grid2(1, 1)
    nb = [[-1, -1, -1, -1, -1, -1]]
    assert A.validate_blocks(2, False, 1.4, p, n, dx, x, nb)[0] == A.OK


def test_product_path_has_no_cpu_fallback():
    # the binding never imports the oracle
    src = open(os.path.join(ROOT, "paper_1407_2052_amd", "amrvac.py")).read()
    assert "oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "paper_1407_2052_amd")):
        if f.endswith(".py"):
            assert "import oracle" not in open(os.path.join(ROOT, "paper_1407_2052_amd", f)).read()


def test_config_struct_layout_matches_header():
    # the binding's Config mirrors amrvac_config field by field
    import ctypes
    src = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} amrvac_config;", src, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"(int|double)\s+(\w+);", body)
    assert [f[1] for f in fields] == [f[0] for f in A.Config._fields_]
    ct = {"int": ctypes.c_int, "double": ctypes.c_double}
    assert [ct[f[0]] for f in fields] == [f[1] for f in A.Config._fields_]
