"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every symbol include/fock.h declares, arguments are rejected before any device
work, and the host BFGS minimiser behaves as a BFGS should."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.optimize

from paper_2606_05297_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fock.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^(?:int|void|const char \*)\s*([a-z_][a-z_0-9]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = lib.load()
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n


def test_version_and_error_text():
    L = lib.load()
    assert L.fock_version() == 1
    rc = L.fock_apply_H(C.byref(lib.ham(3, 1)), None, None, None, None, None, 0, None)
    assert rc == -3 and "d=1" in lib.last_error()


@pytest.mark.parametrize("L_,d,code", [(0, 4, -3), (25, 2, -3), (3, 17, -3), (3, 1, -3), (12, 8, -2), (31, 2, -3)])
def test_geometry_validation(L_, d, code):
    b = C.c_size_t(0)
    assert lib.load().fock_workspace_bytes(C.byref(lib.ham(L_, d)), 0, 0, C.byref(b)) == code


def test_workspace_sizes_grow_with_pool_and_ops():
    h = lib.ham(8, 8, False, 1, 0, 0, 0.5, 0.2)
    a = lib.workspace_bytes(h, 0, 0)
    b = lib.workspace_bytes(h, 28, 0)
    c = lib.workspace_bytes(h, 28, 60)
    assert 0 < a < b < c
    assert c % 256 == 0


def test_argument_validation_before_device_work():
    L = lib.load()
    h = lib.ham(3, 4, False, 1, 2)
    big = C.c_void_p(1 << 20)  # never dereferenced: validation fails first
    # bad op pair (i >= j)
    rc = L.fock_apply_gate2(3, 4, lib.op("HR", 2, 1), 0.1, 0, big, big, 1 << 20, None)
    assert rc == -1 and "i < j" in lib.last_error()
    # out-of-range mode
    rc = L.fock_apply_gate2(3, 4, lib.op("PR", 0, 3), 0.1, 0, big, big, 1 << 20, None)
    assert rc == -1
    # unknown types (the last known one is FOCK_SI = 9)
    for t in (10, 99, -1):
        rc = L.fock_apply_gate2(3, 4, lib.Op(t, 0, 1), 0.1, 0, big, big, 1 << 20, None)
        assert rc == -1 and "unknown" in lib.last_error()
    # non-finite theta
    rc = L.fock_apply_gate2(3, 4, lib.op("HR", 0, 1), float("nan"), 0, big, big, 1 << 20, None)
    assert rc == -4
    # null / misaligned pointers
    rc = L.fock_apply_H(C.byref(h), None, big, None, None, big, 1 << 20, None)
    assert rc == -1 and "psi" in lib.last_error()
    rc = L.fock_apply_H(C.byref(h), C.c_void_p((1 << 20) + 8), big, None, None, big, 1 << 20, None)
    assert rc == -1 and "aligned" in lib.last_error()
    # aliasing
    rc = L.fock_apply_H(C.byref(h), big, big, None, None, big, 1 << 20, None)
    assert rc == -1 and "overlap" in lib.last_error()
    # non-finite Hamiltonian
    hb = lib.ham(3, 4, False, float("inf"), 2)
    assert L.fock_apply_H(C.byref(hb), big, C.c_void_p(2 << 20), None, None, big, 1 << 20, None) == -4
    # pool size limits
    assert L.fock_pool_grads(C.byref(h), lib.ops_array([("HR", 0, 1)]), 5000, big, big, None, big, 0, None) == -1


def test_workspace_too_small_is_reported():
    L = lib.load()
    h = lib.ham(3, 4, False, 1, 2)
    big = C.c_void_p(1 << 20)
    rc = L.fock_apply_H(C.byref(h), big, C.c_void_p(2 << 20), None, None, C.c_void_p(3 << 20), 16, None)
    assert rc == -2 and "workspace" in lib.last_error()
    rc = L.fock_apply_H(C.byref(h), big, C.c_void_p(2 << 20), None, None, C.c_void_p((3 << 20) + 64), 1 << 20, None)
    assert rc == -1 and "256-byte" in lib.last_error()


def test_adapt_create_validation():
    L = lib.load()
    o = lib.AdaptOpts()
    L.adapt_default_opts(C.byref(o))
    assert o.max_iters == 60 and o.bfgs_maxiter == 1000 and o.grad_tol == 1e-3
    st = C.c_void_p()
    h = lib.ham(3, 4, False, 1, 2)
    assert L.adapt_create(C.byref(h), None, 0, C.c_void_p(1 << 20), C.byref(o), None, C.byref(st)) == -1
    o.n_warm = 2  # arrays missing
    assert L.adapt_create(C.byref(h), lib.ops_array([("HR", 0, 1)]), 1, C.c_void_p(1 << 20), C.byref(o), None,
                          C.byref(st)) == -1
    o.n_warm = 0
    o.warm_fixed = 1  # fixed warm-up angles: the complex128 driver only
    assert L.adapt_create(C.byref(h), lib.ops_array([("HR", 0, 1)]), 1, C.c_void_p(1 << 20), C.byref(o), None,
                          C.byref(st)) == -3
    assert not st.value


# ---------------------------------------------------------------- host BFGS

def rosen(x):
    return scipy.optimize.rosen(x), scipy.optimize.rosen_der(x)


def test_bfgs_rosenbrock_reaches_minimum():
    r = lib.bfgs_minimize(rosen, np.array([-1.2, 1.0, 0.5, -0.7]), gtol=1e-9, maxiter=2000)
    assert r["status"] == 0
    assert np.allclose(r["x"], 1.0, atol=1e-6)
    ref = scipy.optimize.minimize(rosen, np.array([-1.2, 1.0, 0.5, -0.7]), jac=True, method="BFGS",
                                  options={"gtol": 1e-9})
    assert abs(r["f"] - ref.fun) < 1e-12


def test_bfgs_quadratic_exact_and_inverse_hessian():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((5, 5))
    A = M @ M.T + 5 * np.eye(5)
    b = rng.standard_normal(5)
    fun = lambda x: (0.5 * x @ A @ x - b @ x, A @ x - b)  # noqa: E731
    r = lib.bfgs_minimize(fun, np.zeros(5), gtol=1e-11, maxiter=200)
    assert np.allclose(r["x"], np.linalg.solve(A, b), atol=1e-9)
    assert r["iters"] <= 15  # quasi-Newton on a 5-dim quadratic with a Wolfe line search
    # the inverse-Hessian estimate approaches A^{-1}
    assert np.abs(r["hinv"] - np.linalg.inv(A)).max() < 0.05
    # recycled inverse Hessian: a second solve from a new start needs fewer iterations
    r2 = lib.bfgs_minimize(fun, np.ones(5), gtol=1e-11, maxiter=200, hinv=r["hinv"])
    r3 = lib.bfgs_minimize(fun, np.ones(5), gtol=1e-11, maxiter=200)
    assert r2["iters"] <= r3["iters"]
    assert np.allclose(r2["x"], np.linalg.solve(A, b), atol=1e-9)


def test_bfgs_reports_objective_errors():
    def bad(x):
        raise ValueError("boom")
    with pytest.raises(Exception):
        lib.bfgs_minimize(bad, np.zeros(2))


def test_stencil_schedules_are_permutations():
    """Every tile schedule visits each tile exactly once and gives every XCD
    (workgroup b runs on XCD b % 8) the same number of tiles; octant schemes
    keep each XCD inside one octant of the three top digits."""
    for (L, d) in [(8, 8), (8, 6), (6, 8), (8, 4), (5, 4), (3, 4)]:
        K = 0
        T = 1
        while K < L - 1 and T * d <= min(4096 // d, 512):
            T *= d
            K += 1
        n = d ** (L - 1) // T
        for s in range(5):
            o = lib.stencil_schedule_table(L, d, s, n)
            assert sorted(o.tolist()) == list(range(n)), (L, d, s)
            if s in (2, 3) and n % 8 == 0 and d % 2 == 0 and n >= 64 and (L - 1 - K) >= 3:
                m = L - 1 - K
                for x in range(8):
                    tiles = o[x::8]
                    digs = [[(t // d ** k) % d for k in range(m)] for t in tiles]
                    key = {(c[m - 1] >= d // 2, c[m - 2] >= d // 2, c[m - 3] >= d // 2) for c in digs}
                    assert len(key) == 1, (L, d, s, x)
    with pytest.raises(lib.FockError):
        lib.set_stencil_schedule(99)


def test_stencil_variant_setter():
    """The H psi work split is a process-wide setting: the three values
    round-trip, anything else is rejected and leaves the setting unchanged; the
    two-pass slab stencil is the default."""
    prev = lib.get_stencil_variant()
    assert prev == lib.STENCIL_SLAB
    try:
        for v in (lib.STENCIL_LANES, lib.STENCIL_SLAB, lib.STENCIL_ROWS):
            lib.set_stencil_variant(v)
            assert lib.get_stencil_variant() == v
        for bad in (3, -1):
            with pytest.raises(lib.FockError):
                lib.set_stencil_variant(bad)
        assert lib.get_stencil_variant() == lib.STENCIL_ROWS
    finally:
        lib.set_stencil_variant(prev)


def test_prof_sample_setter():
    """Event-timing sampling interval: positive values accepted, zero and
    negative rejected; no launch is timed while profiling is off."""
    for v in (4, 1):
        lib.prof_set_sample(v)
    for v in (0, -3):
        with pytest.raises(lib.FockError):
            lib.prof_set_sample(v)
    lib.prof_reset()
    assert lib.prof_query(0)["launches"] == 0


def test_mfma_operand_overlap_check():
    """The build rejects matrix instructions whose destination partially
    overlaps the accumulator input (identical or disjoint ranges are fine)."""
    from paper_2606_05297_amd import build as B
    text = "\n".join([
        "\tv_mfma_f32_16x16x4_f32 a[28:31], v15, v12, a[28:31]",
        "\tv_mfma_f32_16x16x4_f32 a[0:3], v15, v12, a[4:7]",
        "\tv_mfma_f32_16x16x4_f32 a[26:29], v16, v12, a[28:31]",
        "\tv_mfma_f32_16x16x32_bf16 v[4:7], v[0:3], v[8:11], v[4:7]",
        "\tv_mfma_f32_16x16x32_bf16 v[4:7], v[0:3], v[8:11], v[2:5]",
    ])
    n, bad = B.mfma_overlaps(text)
    assert n == 5
    assert bad == ["v_mfma_f32_16x16x4_f32 a[26:29], v16, v12, a[28:31]",
                   "v_mfma_f32_16x16x32_bf16 v[4:7], v[0:3], v[8:11], v[2:5]"]


# ---------------------------------------------------------------- binding argument checks

def test_state_arguments_rejected_before_any_launch():
    """The Python entry points refuse state tensors of the wrong dtype, length
    or device before calling the library (a short or complex128 buffer would
    otherwise be read or written past its end by the kernels)."""
    import torch
    h = lib.ham(3, 4, False, 1, 2)
    good_len = 4 ** 3
    ws = torch.empty(16, dtype=torch.uint8)
    with pytest.raises(lib.FockError, match="complex64"):
        lib.apply_H(h, torch.zeros(good_len, dtype=torch.complex128), torch.zeros(good_len, dtype=torch.complex64), ws)
    with pytest.raises(lib.FockError, match="amplitudes"):
        lib.apply_H(h, torch.zeros(good_len - 1, dtype=torch.complex64), torch.zeros(good_len, dtype=torch.complex64),
                    ws)
    with pytest.raises(lib.FockError, match="GPU"):
        lib.apply_H(h, torch.zeros(good_len, dtype=torch.complex64), torch.zeros(good_len, dtype=torch.complex64), ws)
    with pytest.raises(lib.FockError, match="contiguous"):
        lib.pool_grads(h, [("HR", 0, 1)], torch.zeros(2 * good_len, dtype=torch.complex64)[::2],
                       torch.zeros(good_len, dtype=torch.complex64), ws)
    with pytest.raises(lib.FockError, match="amplitudes"):
        lib.apply_gate2(3, 4, ("HR", 0, 1), 0.1, torch.zeros(good_len + 1, dtype=torch.complex64), ws)
    with pytest.raises(lib.FockError, match="amplitudes"):
        lib.energy_grad_adjoint(h, [("HR", 0, 1)], [0.1], torch.zeros(3, dtype=torch.complex64),
                                torch.zeros(good_len, dtype=torch.complex64), torch.zeros(good_len, dtype=torch.complex64),
                                ws)
    with pytest.raises(lib.FockError, match="complex128"):
        lib.Adapt64(h, [("HR", 0, 1)], torch.zeros(good_len, dtype=torch.complex64))
    with pytest.raises(lib.FockError, match="amplitudes"):
        lib.Adapt(h, [("HR", 0, 1)], torch.zeros(good_len * 4, dtype=torch.complex64))
    with pytest.raises(lib.FockError, match="amplitudes"):
        lib.Sweep([dict(ham=h, pool=[("HR", 0, 1)], psi0=torch.zeros(5, dtype=torch.complex64))])


def test_adapt_create_rejects_oversized_caps():
    L = lib.load()
    o = lib.AdaptOpts()
    L.adapt_default_opts(C.byref(o))
    st = C.c_void_p()
    h = lib.ham(3, 4, False, 1, 2)
    o.max_iters = 1 << 30  # would overflow the workspace's gate count
    assert L.adapt_create(C.byref(h), lib.ops_array([("HR", 0, 1)]), 1, C.c_void_p(1 << 20), C.byref(o), None,
                          C.byref(st)) == -1
    assert "max_iters" in lib.last_error()
    o.max_iters = 60
    o.n_warm = 5000
    wops = lib.ops_array([("HR", 0, 1)] * 5000)
    wth = (C.c_double * 5000)()
    o.warm_ops = C.cast(wops, C.POINTER(lib.Op))
    o.warm_theta0 = C.cast(wth, C.POINTER(C.c_double))
    assert L.adapt_create(C.byref(h), lib.ops_array([("HR", 0, 1)]), 1, C.c_void_p(1 << 20), C.byref(o), None,
                          C.byref(st)) == -1
    assert not st.value


def test_adjoint_sweep_argument_checks():
    L = lib.load()
    h = lib.ham(3, 4, False, 1, 2)
    big = C.c_void_p(1 << 20)
    g = (C.c_double * 2)()
    th = (C.c_double * 2)(0.1, 0.2)
    rc = L.fock_adjoint_sweep(C.byref(h), lib.ops_array([("HR", 0, 1), ("PR", 1, 2)]), th, 2, big, big, 1.0, g, big,
                              1 << 20, None)
    assert rc == -1 and "distinct" in lib.last_error()
    rc = L.fock_adjoint_sweep(C.byref(h), lib.ops_array([("HR", 0, 1), ("PR", 1, 2)]), th, 2, big,
                              C.c_void_p(2 << 20), 0.0, g, C.c_void_p(3 << 20), 1 << 24, None)
    assert rc == -1 and "norm2" in lib.last_error()


def test_apply_H_noalloc_rejects_before_device_work():
    """The allocation-free H psi refuses lattices whose workgroup partials
    exceed its fixed scratch array (L=10, d=8: 262,144 partials) and bad
    pointers, before touching the device."""
    L = lib.load()
    big = lib.ham(10, 8, False, 1.0, 0.0, 0.0, 0.5, 0.2)
    a, b = C.c_void_p(1 << 20), C.c_void_p(2 << 20)
    assert L.fock_apply_H_noalloc(C.byref(big), a, b, None, None) == -2
    assert "scratch" in lib.last_error()
    h = lib.ham(8, 8, False, 1.0, 0.0, 0.0, 0.5, 0.2)
    assert L.fock_apply_H_noalloc(C.byref(h), a, a, None, None) == -1 and "overlap" in lib.last_error()
    assert L.fock_apply_H_noalloc(C.byref(h), None, b, None, None) == -1
    assert L.fock_apply_H_noalloc(C.byref(h), a, b, C.c_void_p((3 << 20) + 4), None) == -1


def test_stream_probe_rejects_before_device_work():
    """The streaming probe validates kind, size, grid, count and pointers
    before it creates events or launches anything."""
    L = lib.load()
    a, b = C.c_void_p(1 << 20), C.c_void_p(2 << 20)
    ms = C.c_double(0.0)
    assert L.fock_stream_probe(3, a, b, 1 << 20, 64, 1, C.byref(ms), None) == -1 and "kind" in lib.last_error()
    assert L.fock_stream_probe(0, a, b, 0, 64, 1, C.byref(ms), None) == -1
    assert L.fock_stream_probe(0, a, b, 24, 64, 1, C.byref(ms), None) == -1
    assert L.fock_stream_probe(0, a, b, 1 << 20, 0, 1, C.byref(ms), None) == -1
    assert L.fock_stream_probe(0, a, b, 1 << 20, 64, 0, C.byref(ms), None) == -1
    assert L.fock_stream_probe(0, None, b, 1 << 20, 64, 1, C.byref(ms), None) == -1
    assert L.fock_stream_probe(2, None, None, 1 << 20, 64, 1, C.byref(ms), None) == -1
    assert L.fock_stream_probe(0, C.c_void_p((1 << 20) + 8), b, 1 << 20, 64, 1, C.byref(ms), None) == -1
    assert L.fock_stream_probe(1, a, b, 64, 64, 1, C.byref(ms), None) == -1 and "too small" in lib.last_error()
    assert L.fock_stream_probe(0, a, b, 1 << 20, 64, 1, None, None) == -1


def test_state_store_switch():
    """The forward-state store defaults to AUTO and takes only OFF, ON, AUTO."""
    L = lib.load()
    assert lib.get_state_store() == lib.STORE_AUTO
    assert L.fock_set_state_store(3) == -1 and "AUTO" in lib.last_error()
    for m in (lib.STORE_OFF, lib.STORE_ON):
        lib.set_state_store(m)
        try:
            assert lib.get_state_store() == m
        finally:
            lib.set_state_store(lib.STORE_AUTO)
    assert lib.get_state_store() == lib.STORE_AUTO


def test_sector_layout_switch_and_argument_checks():
    """The ADAPT sector switch defaults to AUTO and takes only OFF and AUTO; the
    layout field of the Hamiltonian record and the conversions reject bad
    values before any device work (null pointers included)."""
    L = lib.load()
    assert lib.get_sector_layout() == lib.SECTOR_AUTO
    assert L.fock_set_sector_layout(2) == -1 and "AUTO" in lib.last_error()
    lib.set_sector_layout(lib.SECTOR_OFF)
    try:
        assert lib.get_sector_layout() == lib.SECTOR_OFF
    finally:
        lib.set_sector_layout(lib.SECTOR_AUTO)
    assert lib.get_sector_layout() == lib.SECTOR_AUTO
    nb = C.c_size_t(0)
    # layout outside {0, 1, 2}; halved layout off the supported chains
    for h in (lib.ham(8, 8, layout=3), lib.ham(8, 6, layout=1), lib.ham(8, 8, periodic=True, layout=2),
              lib.ham(6, 8, layout=1)):
        assert L.fock_workspace_bytes(C.byref(h), 0, 0, C.byref(nb)) in (-1, -3)
    h = lib.ham(8, 8, layout=lib.LAYOUT_EVEN)
    assert L.fock_workspace_bytes(C.byref(h), 28, 20, C.byref(nb)) == 0 and nb.value > 0
    # calls that take full states only
    assert L.fock_apply_H_noalloc(C.byref(h), None, None, None, None) in (-1, -3)
    # conversions: d, layout and pointers checked first
    assert L.fock_sector_pack(8, 6, 1, None, None, None) == -3
    assert L.fock_sector_pack(8, 8, 0, None, None, None) == -1
    assert L.fock_sector_unpack(8, 8, 1, None, None, None) == -1


def test_real_fusion_switch():
    """Fused runs of real gates default to ON and the switch takes only OFF
    and ON."""
    L = lib.load()
    assert lib.get_real_fusion() == lib.RFUSE_ON
    assert L.fock_set_real_fusion(2) == -1 and "ON" in lib.last_error()
    lib.set_real_fusion(lib.RFUSE_OFF)
    try:
        assert lib.get_real_fusion() == lib.RFUSE_OFF
    finally:
        lib.set_real_fusion(lib.RFUSE_ON)
    assert lib.get_real_fusion() == lib.RFUSE_ON


def _runs_from_definition(ops, top, on=True):
    """Greedy runs written from their definition: extend while every pair of
    the run lies in one window of three consecutive modes at or below `top`
    (at most 8 gates); a run of one gate is a single gate (-1)."""
    runs, k, n = [], 0, len(ops)
    ok = [on and o[2] == o[1] + 1 and o[2] <= top for o in ops]
    while k < n:
        m = k + 1
        if ok[k]:
            lo = hi = ops[k][1]
            while m < n and m - k < 8 and ok[m] and max(hi, ops[m][1]) - min(lo, ops[m][1]) <= 1:
                lo, hi = min(lo, ops[m][1]), max(hi, ops[m][1])
                m += 1
        if m - k >= 2:
            a = min(lo, top - 2)
            assert a <= lo and hi + 1 <= a + 2 and a >= 0
            runs.append((k, a))
        else:
            runs.append((k, -1))
            m = k + 1
        k = m
    return runs


def test_real_fusion_plan():
    """The run planner of real-state evaluations (host only): the benchmark's
    ansatz, the top pair of the parity-halved layout left single, the top
    window of the full layout, runs split at 8 gates, small states unfused,
    fusion switched off; every run's pairs inside its tile's three modes."""
    bench = [("PR", b, b + 1) for b in range(7)] + [("HR", 0, 1), ("PR", 1, 2), ("PR", 0, 1), ("PR", 2, 3),
                                                     ("HR", 2, 3), ("HR", 1, 2), ("PR", 1, 2), ("PR", 2, 3),
                                                     ("PR", 3, 4), ("HR", 3, 4), ("PR", 3, 4), ("PR", 4, 5),
                                                     ("HR", 4, 5)]
    mixed = [("PR", 5, 6), ("PR", 6, 7), ("HR", 5, 6)] + [("HR", 3, 4)] * 10 + [("PR", 0, 1)]
    halved, full = lib.ham(8, 8, layout=lib.LAYOUT_EVEN | lib.LAYOUT_REAL), lib.ham(8, 8, layout=lib.LAYOUT_REAL)
    for h, top in ((halved, 6), (full, 7)):
        for ops in (bench, mixed, [], [("HR", 2, 3)]):
            got = lib.real_fusion_plan(h, ops)
            assert got == _runs_from_definition(ops, top), (top, ops, got)
            bounds = [r[0] for r in got] + [len(ops)]
            for (k0, a), k1 in zip(got, bounds[1:]):
                if a >= 0:
                    assert k1 - k0 >= 2 and all(a <= o[1] and o[2] <= a + 2 for o in ops[k0:k1])
    assert lib.real_fusion_plan(halved, bench) == [(0, 0), (2, 2), (4, 4), (6, -1), (7, 0), (10, 1), (15, 3)]
    # the top pair joins a run only in the full layout
    assert lib.real_fusion_plan(halved, mixed)[:2] == [(0, -1), (1, -1)]
    assert lib.real_fusion_plan(full, mixed)[0] == (0, 5)
    # states below 2^21 stored amplitudes, and fusion off: every gate by itself
    small = lib.ham(6, 8)
    assert lib.real_fusion_plan(small, bench[:5]) == [(k, -1) for k in range(5)]
    lib.set_real_fusion(lib.RFUSE_OFF)
    try:
        assert lib.real_fusion_plan(halved, bench) == [(k, -1) for k in range(len(bench))]
    finally:
        lib.set_real_fusion(lib.RFUSE_ON)
    with pytest.raises(lib.FockError):
        lib.real_fusion_plan(halved, [("HI", 0, 1)])
    with pytest.raises(lib.FockError):
        lib.real_fusion_plan(halved, [("HR", 0, 8)])


def test_prepare_rejects_bad_geometry():
    """fock_prepare checks (L, d) like the other calls before touching a device."""
    L = lib.load()
    assert L.fock_prepare(0, 8) == -3
    assert L.fock_prepare(8, 1) == -3
    assert L.fock_prepare(12, 16) == -2  # d^L beyond 2^31 amplitudes
