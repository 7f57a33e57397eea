"""The C-ABI library loads on the CPU and exports every entry point that
include/ns.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ns.h")
LIB = os.path.join(ROOT, "paper_1810_10197_amd", "libns.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ns_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libns.so not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "ns_init" in names and "ns_step_bs5" in names and "ns_integrate" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    from paper_1810_10197_amd import ns
    assert sorted(ns.EXPORTS) == declared()


def test_host_only_entry_points(lib):
    from paper_1810_10197_amd import ns
    ok = ns.NsConfig(3, 32, 1, 0, 0, 0.0, 0.0, 0.0, 0.0)
    assert ns.ns_workspace_bytes(ok) > 0
    assert ns.ns_workspace_bytes(ns.NsConfig(2, 1024, 1, 0, 1, 0.5, 1e-4, 0, 0)) > 0
    assert ns.ns_workspace_bytes(ns.NsConfig(2, 64, 3, 1, 0, 0, 0, 0, 0)) > 0
    w1024 = ns.ns_workspace_bytes(ns.NsConfig(3, 1024, 1, 0, 0, 0, 0, 0, 0))
    assert 150e9 < w1024 < 200e9              # fits the 288 GB of one MI355X
    assert ns.ns_workspace_bytes(ns.NsConfig(2, 1024, 1, 0, 1, 0.5, 1e-4, 0, 0, 1)) > 0   # 3/2 rule
    for bad in [ns.NsConfig(3, 48, 1, 0, 0, 0, 0, 0, 0),     # not a power of two
                ns.NsConfig(3, 2048, 1, 0, 0, 0, 0, 0, 0),   # limited to 1024
                ns.NsConfig(3, 1024, 1, 0, 0, 0, 0, 0, 0, 1),  # 3/2 rule: 3D up to 512
                ns.NsConfig(4, 32, 1, 0, 0, 0, 0, 0, 0),
                ns.NsConfig(3, 32, 0, 0, 0, 0, 0, 0, 0),
                ns.NsConfig(3, 32, 1, 2, 0, 0, 0, 0, 0),
                ns.NsConfig(3, 32, 1, 0, 1, 0, 0, 0, 0),     # scalar needs 2D
                ns.NsConfig(2, 2048, 1, 0, 1, 0, 0, 0, 0),   # 2D limited to 1024
                ns.NsConfig(3, 32, 1, 0, 0, 0, 0, 0, 0, 2),  # no such dealiasing rule
                ns.NsConfig(3, 8, 1, 0, 0, 0, 0, 0, 0, 1)]:  # 3/2 rule: n >= 16
        assert ns.ns_workspace_bytes(bad) == 0
    assert ns.ns_strerror(ns.NS_ERR_STEPFAIL).startswith("too many")
    # argument errors are caught before any device call
    h = ctypes.c_void_p()
    nu = (ctypes.c_double * 1)(0.01)
    rc = lib.ns_init(ctypes.byref(ok), nu, ctypes.c_void_p(0), ctypes.c_size_t(0),
                     ctypes.c_void_p(0), ctypes.byref(h))
    assert rc == ns.NS_ERR_ARG


def test_workspace_scales_with_problem():
    from paper_1810_10197_amd import ns
    a = ns.ns_workspace_bytes(ns.NsConfig(3, 128, 1, 0, 0, 0, 0, 0, 0))
    b = ns.ns_workspace_bytes(ns.NsConfig(3, 128, 4, 0, 0, 0, 0, 0, 0))
    c = ns.ns_workspace_bytes(ns.NsConfig(3, 128, 1, 1, 0, 0, 0, 0, 0))
    assert 3.5 * a < b < 4.5 * a
    assert c > a
    # the 3/2 rule keeps (n-1)^2 n/2 modes (not ~(2n/3)^2 n/3) and forms the
    # products on the (3n/2)^3 grid: its workspace is several times larger
    d = ns.ns_workspace_bytes(ns.NsConfig(3, 128, 1, 0, 0, 0, 0, 0, 0, 1))
    assert d > 3 * a
