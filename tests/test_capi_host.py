"""C-ABI checks that need no GPU: the library loads, exports every declared symbol, and
validates arguments / call order on a host-only context (no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2405_05213_amd import ep as epmod
from workloads import config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ep.h")).read()
    return sorted(set(re.findall(r"^(?:ep_status|const char\*)\s+(ep_\w+)\(", src, flags=re.M)))


def test_header_and_binding_agree():
    assert _declared() == epmod.EXPORTED


def test_library_exports_every_declared_symbol():
    L = epmod.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert b"gfx950" in L.ep_version()


def _host_ctx():
    return epmod.Context(device=-1)


def test_validation_errors():
    c = _host_ctx()
    p = config("c1")
    with pytest.raises(epmod.EPError) as e:
        c.set_mesh(p.xyz, p.conn + 1000)
    assert e.value.code == epmod.EP_ERR_ARG
    c.set_mesh(p.xyz, p.conn)
    with pytest.raises(epmod.EPError) as e:
        c.set_material("linear", (200e9, 0.7), 7800.0)
    assert e.value.code == epmod.EP_ERR_ARG
    with pytest.raises(epmod.EPError):
        c.set_material("yeoh", (1.0, 0.0, 0.0), 1000.0)
    with pytest.raises(epmod.EPError):
        c.set_dirichlet([3 * p.n_nodes])
    with pytest.raises(epmod.EPError):
        c.set_traction(p.faces, p.t0, [0.0, 0.0], [1.0, 2.0])       # knots not ascending
    with pytest.raises(epmod.EPError):
        c.set_krylov(m_max=300)
    with pytest.raises(epmod.EPError):
        c.set_krylov(m_fixed=70, m_max=64)
    # order: state / step before binding
    with pytest.raises(epmod.EPError) as e:
        c.step(1e-4)
    assert e.value.code == epmod.EP_ERR_ORDER
    with pytest.raises(epmod.EPError) as e:
        c.workspace_size()                     # material missing
    assert e.value.code == epmod.EP_ERR_ORDER
    c.set_material("linear", (200e9, 0.3), 7800.0)
    assert c.workspace_size() > 0


def test_workspace_size_scales_with_subspace():
    p = config("c1")
    sizes = []
    for m in (16, 64):
        c = _host_ctx()
        c.set_mesh(p.xyz, p.conn)
        c.set_material("linear", (200e9, 0.3), 7800.0)
        c.set_krylov(m_max=m)
        sizes.append(c.workspace_size())
    assert sizes[1] > sizes[0]


def test_host_context_cannot_bind():
    L = epmod.lib()
    c = _host_ctx()
    p = config("c1")
    c.set_mesh(p.xyz, p.conn)
    c.set_material("linear", (200e9, 0.3), 7800.0)
    n = c.workspace_size()
    rc = L.ep_bind_workspace(c.h, C.c_void_p(256), n)
    assert rc == epmod.EP_ERR_HIP
    rc = L.ep_bind_workspace(c.h, C.c_void_p(257), n)
    assert rc == epmod.EP_ERR_WORKSPACE


def test_orthogonalization_modes():
    """Compact-WY MGS is the default up to m_max = 64; larger subspaces use the sequential
    form; an explicit compact-WY request beyond 64 is refused."""
    p = config("c1")

    def ctx(m_max, mode=None):
        c = _host_ctx()
        c.set_mesh(p.xyz, p.conn)
        c.set_material("linear", (200e9, 0.3), 7800.0)
        c.set_krylov(m_max=m_max)
        if mode is not None:
            c.set_orthogonalization(mode)
        return c

    assert ctx(64).orthogonalization() == 1
    assert ctx(65).orthogonalization() == 0
    assert ctx(64, 0).orthogonalization() == 0
    c = ctx(128, 1)
    with pytest.raises(epmod.EPError) as e:
        c.workspace_size()
    assert e.value.code == epmod.EP_ERR_ARG
    with pytest.raises(epmod.EPError) as e:
        _host_ctx().set_orthogonalization(2)
    assert e.value.code == epmod.EP_ERR_ARG
    # the vector all-reduce slots make the compact-WY workspace larger
    assert ctx(64, 1).workspace_size() >= ctx(64, 0).workspace_size()


def test_precision_modes():
    """The BF16-tangent mode reserves its stored tangents (1152 bytes per element, groups of
    8 elements) in the workspace; unknown modes are refused, and batches take only the FP64
    and FP32 modes."""
    p = config("c3", nx=9, ny=2, nz=2)

    def size(prec):
        c = _host_ctx()
        c.set_mesh(p.xyz, p.conn)
        c.set_material("nh", (0.4e6, 2e6), 1100.0)
        c.set_precision(prec)
        return c.workspace_size()

    n_e = p.conn.shape[0]
    assert size("mixed_f32") == size("f64")
    assert size("mixed_bf16") - size("f64") >= 1152 * 8 * ((n_e + 7) // 8)
    L = epmod.lib()
    c = _host_ctx()
    assert L.ep_set_precision(c.h, 3) == epmod.EP_ERR_ARG
    b = epmod.Batch(device=-1)
    b.set_precision("mixed_bf16")               # before the first instance: refused at sizing
    b.add(config("c3", nx=20, ny=4, nz=4))
    with pytest.raises(epmod.EPError) as e:
        b.workspace_size()
    assert e.value.code == epmod.EP_ERR_ARG
    assert L.ep_set_precision(b.h, 2) == epmod.EP_ERR_ARG
    assert L.ep_set_precision(b.h, 1) == epmod.EP_OK
    assert b.workspace_size() > 0


def test_scheme_arguments():
    """ep_set_scheme takes 2 or 4, before binding."""
    c = _host_ctx()
    for order in (0, 1, 3, 6):
        with pytest.raises(epmod.EPError) as e:
            c.set_scheme(order)
        assert e.value.code == epmod.EP_ERR_ARG
    c.set_scheme(4)
    c.set_scheme(2)
