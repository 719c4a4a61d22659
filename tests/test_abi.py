"""The C-ABI library loads and exports every symbol include/slpic.h declares
(no compute calls: this runs without a GPU), and the host-side planning
validates configurations."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(slpic(?:2d)?_\w+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import torch  # noqa: F401  (the library shares torch's HIP runtime)
    from paper_1511_08225_amd import slpic
    L = slpic.lib()
    names = _declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_workspace_planning_validates_configs():
    import torch  # noqa: F401
    import workloads
    from paper_1511_08225_amd import slpic
    L = slpic.lib()
    good = slpic.run_config(workloads.small_sheath())
    t = slpic.tuning("f64")
    n = L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(t))
    assert n > 0
    # more particles need more bytes; F64 more than F32
    big = slpic.run_config(workloads.small_sheath(ppc=200))
    assert L.slpic_workspace_bytes(ctypes.byref(big), 1, ctypes.byref(t)) > n
    t32 = slpic.tuning("f32")
    assert L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(t32)) < n
    for bad in ({"nx": 2}, {"dx": 0.0}, {"dt": -1.0}, {"source_cells": 0}, {"u": 0.0},
                {"beta_kind": 7}):
        cfg = workloads.small_sheath()
        cfg.update(bad)
        c = slpic.run_config(cfg)
        assert L.slpic_workspace_bytes(ctypes.byref(c), 1, ctypes.byref(t)) == 0, bad
    assert L.slpic_workspace_bytes(ctypes.byref(good), 0, ctypes.byref(t)) == 0
    tb = slpic.tuning("f32", block=100)
    assert L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(tb)) == 0
    for order, ok in ((0, True), (1, True), (2, False), (-1, False)):
        to = slpic.tuning("f32", push_order=order)
        assert (L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(to)) > 0) == ok, order
    # recording the sort permutation: 0 or 1 (the buffer is kept either way: a
    # speed-limit change uses it)
    for rp, ok in ((0, True), (1, True), (2, False), (-1, False)):
        tr = slpic.tuning("f32")
        tr.record_perm = rp
        assert (L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(tr)) > 0) == ok, rp
    # sort tiles of at most 32768 slots (the scatter's per-wave offsets are 16-bit)
    for st, ok in ((32768, True), (512, True), (32769, False), (65536, False)):
        ts = slpic.tuning("f32", sort_tile=st)
        assert (L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(ts)) > 0) == ok, st
    inf = slpic.run_config(workloads.sheath(nx=64, ppc=10, u_over_vti=math.inf))
    assert L.slpic_workspace_bytes(ctypes.byref(inf), 1, ctypes.byref(t)) > 0


def test_strerror():
    import torch  # noqa: F401
    from paper_1511_08225_amd import slpic
    L = slpic.lib()
    assert L.slpic_strerror(0) == b"ok"
    assert b"workspace" in L.slpic_strerror(-2)
    assert L.slpic_strerror(12345) == b"unknown error"


def test_init_rejects_bad_workspace_without_touching_gpu():
    import torch  # noqa: F401
    import workloads
    from paper_1511_08225_amd import slpic
    L = slpic.lib()
    c = slpic.run_config(workloads.small_sheath())
    t = slpic.tuning("f64")
    ctx = ctypes.c_void_p()
    # misaligned workspace pointer and a too-small workspace are refused before any HIP call
    rc = L.slpic_init(ctypes.byref(c), 1, ctypes.byref(t), ctypes.c_void_p(8), 1 << 30, None,
                      ctypes.byref(ctx))
    assert rc == -1 and not ctx.value
    rc = L.slpic_init(ctypes.byref(c), 1, ctypes.byref(t), ctypes.c_void_p(1 << 20), 16, None,
                      ctypes.byref(ctx))
    assert rc == -2 and not ctx.value


def test_2d_workspace_planning_validates_configs():
    import torch  # noqa: F401
    import workloads
    from paper_1511_08225_amd import slpic
    L = slpic.lib()
    cfg = workloads.sheath2d(nx=64, ny=64, ppc=4)
    good = slpic.run_config(cfg)
    t = slpic.Tuning2D()
    n = L.slpic2d_workspace_bytes(ctypes.byref(good), 64, ctypes.byref(t))
    assert n > 0
    assert "slpic2d_step" in _declared_functions()
    # ny must be a power of two in [4, 2048]
    for ny in (3, 48, 4096):
        assert L.slpic2d_workspace_bytes(ctypes.byref(good), ny, ctypes.byref(t)) == 0, ny
    # too many sort blocks for the LDS histogram, bad tile/per_thread values
    for field, val in (("tile", 100), ("per_thread", 3), ("margin", 40), ("precision", 5)):
        tb = slpic.Tuning2D()
        setattr(tb, field, val)
        assert L.slpic2d_workspace_bytes(ctypes.byref(good), 64, ctypes.byref(tb)) == 0, field
    # sort tiles: multiples of 1024 up to 32768 slots (the scatter's per-wave
    # offsets within a tile are 16-bit)
    for val, ok in ((32768, True), (2048, True), (65536, False), (1536, False)):
        tb = slpic.Tuning2D()
        tb.sort_tile = val
        assert (L.slpic2d_workspace_bytes(ctypes.byref(good), 64, ctypes.byref(tb)) > 0) == ok, val
    big = slpic.run_config(workloads.sheath2d(nx=2048, ny=2048, ppc=1))
    tb = slpic.Tuning2D()
    tb.tile = 16  # 128 x 128 = 16384 blocks > 4096
    assert L.slpic2d_workspace_bytes(ctypes.byref(big), 2048, ctypes.byref(tb)) == 0
    # the sort permutation: 0 or 1, and its 4 B per slot only when recorded
    for rp, ok in ((0, True), (1, True), (2, False)):
        tb = slpic.Tuning2D()
        tb.record_perm = rp
        assert (L.slpic2d_workspace_bytes(ctypes.byref(good), 64, ctypes.byref(tb)) > 0) == ok, rp
    tb = slpic.Tuning2D()
    tb.record_perm = 1
    assert L.slpic2d_workspace_bytes(ctypes.byref(good), 64, ctypes.byref(tb)) >= n + 4 * 64 * 64 * 4 * 2
    # F64 needs more bytes than F32
    t64 = slpic.Tuning2D()
    t64.precision = slpic.SLPIC_F64
    assert L.slpic2d_workspace_bytes(ctypes.byref(good), 64, ctypes.byref(t64)) > n


def test_plates_planning_validates_configs():
    """The plates geometry plans like a sheath run sized on the load density
    (its box starts empty); it rejects warm profiles, more than 16384 cells,
    a non-finite bias, an unknown geometry and the 2D library."""
    import torch  # noqa: F401
    import numpy as np
    import workloads
    from paper_1511_08225_amd import slpic
    L = slpic.lib()
    t = slpic.tuning(precision="f64", sort_every=1)
    cfg = workloads.plates_sheath(0.0158, ppc=40)
    good = slpic.run_config(cfg)
    assert good.geometry == slpic.GEOM_PLATES and good.bias == cfg["bias"]
    n_pl = L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(t))
    sh = slpic.run_config(dict(cfg, geometry="sheath"))
    assert n_pl > 0 and n_pl == L.slpic_workspace_bytes(ctypes.byref(sh), 1, ctypes.byref(t))
    prof = np.zeros((5, 256))
    bad = slpic.run_config(cfg)
    bad.warm_profile = prof.ctypes.data
    assert L.slpic_workspace_bytes(ctypes.byref(bad), 1, ctypes.byref(t)) == 0
    for field, val in (("geometry", 3), ("bias", float("nan")), ("nx", 16385)):
        bad = slpic.run_config(cfg)
        setattr(bad, field, val)
        assert L.slpic_workspace_bytes(ctypes.byref(bad), 1, ctypes.byref(t)) == 0, field
    assert L.slpic2d_workspace_bytes(ctypes.byref(good), 64, ctypes.byref(slpic.Tuning2D())) == 0
    assert "slpic_set_flux_counters" in _declared_functions()
    # the longest run: 2729 cells
    edge = slpic.run_config(dict(workloads.sheath(nx=2729, ppc=2, u_over_vti=3.0), sort_every=1))
    assert L.slpic_workspace_bytes(ctypes.byref(edge), 1, ctypes.byref(t)) > 0
    edge.nx = 2730
    assert L.slpic_workspace_bytes(ctypes.byref(edge), 1, ctypes.byref(t)) == 0


def test_periodic_planning_validates_configs():
    import torch  # noqa: F401
    import numpy as np
    import workloads
    from paper_1511_08225_amd import slpic
    L = slpic.lib()
    t = slpic.tuning(precision="f32", sort_every=16)
    cfg = workloads.langmuir_box(0.25, nx=256, ppc=10)
    good = slpic.run_config(cfg)
    assert good.geometry == slpic.GEOM_PERIODIC
    assert L.slpic_workspace_bytes(ctypes.byref(good), 1, ctypes.byref(t)) > 0
    big = slpic.run_config(dict(cfg, nx=16385))
    assert L.slpic_workspace_bytes(ctypes.byref(big), 1, ctypes.byref(t)) == 0
    prof = np.zeros((5, 256))
    warm = slpic.run_config(cfg)
    warm.warm_profile = prof.ctypes.data
    assert L.slpic_workspace_bytes(ctypes.byref(warm), 1, ctypes.byref(t)) == 0
