"""The C interface on the host: library loads, every declared symbol is
exported, and the host-only logic (stability bound, eq.(alpha), argument
checks, weight folding) matches the oracle.  No GPU work is issued."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import synthetic as S
from oracle import fdtd as O
from paper_1710_06829_amd import _binding as B
import paper_1710_06829_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(xfdtd_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    # and the binding wraps exactly these
    assert set(names) <= set(B.SIGNATURES), set(names) - set(B.SIGNATURES)


def test_abi_version():
    assert B.lib().xfdtd_abi_version() >= 1


@pytest.mark.parametrize("seed", range(10))
def test_cfl_limit_matches_oracle(seed):
    g = S.rng(3000 + seed)
    beta = g.uniform(-0.05, 0.2, (3, 2))
    delta = g.uniform(-0.2, 0.05, 3)
    c = O.coeffs_from(beta, delta)
    d = tuple(g.uniform(0.5, 2.0, 3))
    dtm, fmn, fmx = pkg.cfl_limit((4, 4, 4), c, d)
    omn, omx = O.stability_range(c, d)
    assert abs(fmx - omx) < 1e-12 * abs(omx)
    assert abs(fmn - omn) < 1e-12 * max(1.0, abs(omx))
    assert abs(dtm - 1 / np.sqrt(omx)) < 1e-12


def test_consistent_alpha():
    beta, delta = S.distinct_beta_delta(5)
    c = O.coeffs_from(beta, delta)
    raw = c.copy()
    raw[[0, 4, 8]] = 7.0
    assert np.allclose(pkg.consistent_alpha(raw), c, atol=1e-15, rtol=0)


def _create(shape=(4, 5, 6), dt=0.3, coeffs=None, dtype=B.XFDTD_F64, allow=0, spacing=(1, 1, 1)):
    g = B.make_grid(shape, spacing)
    h = ctypes.c_void_p()
    c = O.yee_coeffs() if coeffs is None else coeffs
    rc = B.lib().xfdtd_create(ctypes.byref(g), dt, B.dbl_array(c, 12), dtype, allow, ctypes.byref(h))
    return rc, h


def test_create_rejects_unstable_dt_and_bad_arguments():
    beta, delta = S.extended_beta_delta(6)
    c = O.coeffs_from(beta, delta)
    cfl = O.cfl_dt(c)
    rc, h = _create(dt=cfl * 1.001, coeffs=c)
    assert rc == -2 and not h.value
    assert b"stability" in B.lib().xfdtd_last_error()
    rc, h = _create(dt=cfl * 1.001, coeffs=c, allow=1)
    assert rc == 0
    B.lib().xfdtd_destroy(h)
    rc, h = _create(dt=cfl * 0.999, coeffs=c)
    assert rc == 0
    B.lib().xfdtd_destroy(h)
    assert _create(shape=(0, 4, 4))[0] == -1
    assert _create(dt=-1.0)[0] == -1
    assert _create(dt=float("nan"))[0] == -1
    assert _create(dtype=3)[0] == -1
    assert _create(spacing=(1, 0, 1))[0] == -1
    # z-planes are limited to 2^28 cells (32-bit plane offsets in the kernels)
    assert _create(shape=(1, 1 << 14, 1 << 15))[0] == -1
    rc, h = _create(shape=(1, 1 << 14, 1 << 14))
    assert rc == 0
    B.lib().xfdtd_destroy(h)
    bad = O.yee_coeffs()
    bad[5] = float("inf")
    assert _create(coeffs=bad)[0] == -1
    # F_min < 0 (strongly negative delta) is rejected as ill-defined
    neg = O.coeffs_from([[0.5, 0.5], [0.0, 0.0], [0.0, 0.0]], [0.0, 0.0, 0.0])
    assert O.stability_range(neg)[0] < 0
    assert _create(dt=0.01, coeffs=neg)[0] == -2


def test_alpha_warning_flag():
    c = O.yee_coeffs()
    rc, h = _create(coeffs=c)
    assert rc == 0 and B.lib().xfdtd_flags(h) == 0
    B.lib().xfdtd_destroy(h)
    c[0] = 0.9
    rc, h = _create(coeffs=c, dt=0.2)
    assert rc == 0 and B.lib().xfdtd_flags(h) & B.WARN_ALPHA
    B.lib().xfdtd_destroy(h)


@pytest.mark.parametrize("dtype,npdt", [(B.XFDTD_F32, np.float32), (B.XFDTD_F64, np.float64)])
def test_weight_folding(dtype, npdt):
    beta, delta = S.distinct_beta_delta(8)
    c = O.coeffs_from(beta, delta)
    sp = (1.0, 0.7, 1.3)
    dt = 0.9 * O.cfl_dt(c, sp)
    rc, h = _create(coeffs=c, dt=dt, dtype=dtype, spacing=sp)
    assert rc == 0
    w = (ctypes.c_double * 15)()
    nw = ctypes.c_int()
    assert B.lib().xfdtd_get_weights(h, w, ctypes.byref(nw)) == 0 and nw.value == 15
    B.lib().xfdtd_destroy(h)
    for a in range(3):
        s = dt / sp[a]
        exp = [s * (c[4 * a] + c[4 * a + 3]), s * c[4 * a + 3], s * c[4 * a + 1], s * c[4 * a + 2], s]
        for m in range(5):
            assert w[5 * a + m] == float(npdt(exp[m]))


@pytest.mark.parametrize("nx,tx", [(96, 32), (32, 32), (80, 32), (5, 32), (48, 64), (128, 64), (160, 64),
                                   (512, 64)])
def test_default_tile_width(nx, tx):
    """Untuned default: 32-column tiles for boxes at most 96 wide that they
    cover with fewer loaded columns (tile plus four halo columns)."""
    rc, h = _create(shape=(8, 8, nx))
    assert rc == 0
    v = [ctypes.c_int() for _ in range(4)]
    assert B.lib().xfdtd_launch_config(h, *[ctypes.byref(x) for x in v]) == 0
    assert v[0].value == tx
    assert v[3].value == -(-nx // tx) * -(-8 // v[1].value) * -(-8 // v[2].value)
    B.lib().xfdtd_destroy(h)


@pytest.mark.parametrize("shape", [(96, 96, 96), (128, 128, 128), (256, 256, 512), (192, 192, 352), (9, 40, 70),
                                   (300, 8, 8), (32, 32, 32), (64, 64, 64)])
def test_default_zchunk_minimises_round_cost(shape):
    """Without a device the library assumes 256 CUs with one resident
    workgroup each; the default z-chunk of the one-step kernel then minimises
    rounds x (z + 3) over the balanced chunk lengths ceil(nz / c), down to
    one plane (a box too small to fill the CUs takes short chunks), checked
    by brute force over every chunk count c."""
    rc, h = _create(shape=shape)
    assert rc == 0
    v = [ctypes.c_int() for _ in range(4)]
    assert B.lib().xfdtd_launch_config(h, *[ctypes.byref(x) for x in v]) == 0
    B.lib().xfdtd_destroy(h)
    tx, ty, zc = v[0].value, v[1].value, v[2].value
    nz, ny, nx = shape
    tiles = -(-nx // tx) * -(-ny // ty)

    def cost(z):
        return -(-tiles * -(-nz // z) // 256) * (z + 3)

    zs = [-(-nz // c) for c in range(1, nz + 1)]
    assert cost(zc) == min(cost(z) for z in zs)


def test_calls_without_bound_fields_are_state_errors():
    rc, h = _create()
    assert rc == 0
    assert B.lib().xfdtd_run(h, 3) == -5
    assert B.lib().xfdtd_step_faraday(h) == -5
    assert B.lib().xfdtd_tune(h, 0, None) == -5
    out = (ctypes.c_double * 3)()
    assert B.lib().xfdtd_divergence_max(h, None, None, out) == -5
    B.lib().xfdtd_destroy(h)
    assert B.lib().xfdtd_run(None, 1) == -1


def test_bind_checks_pointers_before_any_device_call():
    rc, h = _create(shape=(4, 4, 4))
    assert rc == 0
    nbytes = 64 * 8
    base = 1 << 40
    f = (ctypes.c_void_p * 6)(*[base + i * nbytes for i in range(6)])
    f_overlap = (ctypes.c_void_p * 6)(*[base + i * (nbytes // 2) for i in range(6)])
    f_misaligned = (ctypes.c_void_p * 6)(*[base + 8 + i * nbytes for i in range(6)])
    f_null = (ctypes.c_void_p * 6)(*[base + i * nbytes if i != 3 else 0 for i in range(6)])
    assert B.lib().xfdtd_bind(h, f_overlap, None, None) == -1
    assert B.lib().xfdtd_bind(h, f_misaligned, None, None) == -1
    assert B.lib().xfdtd_bind(h, f_null, None, None) == -1
    s_overlap = (ctypes.c_void_p * 6)(*[base + 3 * nbytes + i * nbytes for i in range(6)])
    assert B.lib().xfdtd_bind(h, f, s_overlap, None) == -1
    assert B.lib().xfdtd_bind(h, None, None, None) == -1
    B.lib().xfdtd_destroy(h)


def test_package_has_no_cpu_fallback():
    """The GPU entry points refuse CPU tensors instead of computing on the host."""
    import torch
    f = [torch.zeros((4, 4, 4), dtype=torch.float64) for _ in range(6)]
    with pytest.raises(ValueError):
        pkg.Solver(f, 0.3, O.yee_coeffs())
    with pytest.raises(ValueError):
        pkg.dispersion(torch.zeros((3, 3), dtype=torch.float64), 0.3, O.yee_coeffs())


def test_batch_create_validates_every_box():
    beta, delta = S.extended_beta_delta(9)
    c = O.coeffs_from(beta, delta)
    dt = 0.9 * O.cfl_dt(c)
    grids = (B.Grid * 3)(B.make_grid((4, 5, 6)), B.make_grid((8, 8, 8)), B.make_grid((3, 2, 1)))
    dts = (ctypes.c_double * 3)(dt, dt, dt)
    cc = (ctypes.c_double * 36)(*(list(c) * 3))
    h = ctypes.c_void_p()
    assert B.lib().xfdtd_batch_create(grids, dts, cc, 3, B.XFDTD_F32, 0, ctypes.byref(h)) == 0
    B.lib().xfdtd_batch_destroy(h)
    bad = (ctypes.c_double * 3)(dt, dt * 1.2, dt)
    assert B.lib().xfdtd_batch_create(grids, bad, cc, 3, B.XFDTD_F32, 0, ctypes.byref(h)) == -2
    assert b"box 1" in B.lib().xfdtd_last_error()
    assert B.lib().xfdtd_batch_create(grids, bad, cc, 3, B.XFDTD_F32, 1, ctypes.byref(h)) == 0
    # calls before binding are state errors; bad configurations are rejected
    assert B.lib().xfdtd_batch_run(h, 2) == -5
    assert B.lib().xfdtd_batch_tune(h, 0, None) == -5
    assert B.lib().xfdtd_batch_set_config(h, 64, 5, 1, 0) == -1
    assert B.lib().xfdtd_batch_set_config(h, 64, 4, -1, 0) == -1
    assert B.lib().xfdtd_batch_set_config(h, 64, 4, 0, 0) == 0  # 0: per-box z-chunks from the model
    assert B.lib().xfdtd_batch_set_config(h, 48, 4, 1, 0) == -1
    assert B.lib().xfdtd_batch_set_config(h, 64, 4, 2, 0) == 0
    assert B.lib().xfdtd_batch_set_config(h, 32, 16, 1, 0) == 0
    tx, ty = ctypes.c_int(), ctypes.c_int()
    assert B.lib().xfdtd_batch_get_config(h, ctypes.byref(tx), ctypes.byref(ty), None, None, None) == 0
    assert (tx.value, ty.value) == (32, 16)
    B.lib().xfdtd_batch_destroy(h)
    g0 = (B.Grid * 1)(B.make_grid((0, 5, 6)))
    assert B.lib().xfdtd_batch_create(g0, dts, cc, 1, B.XFDTD_F32, 0, ctypes.byref(h)) == -1
    assert B.lib().xfdtd_batch_create(grids, dts, cc, 0, B.XFDTD_F32, 0, ctypes.byref(h)) == -1


def test_adjoint_step_rejects_aliased_arrays_before_device_work():
    rc, h = _create(shape=(4, 4, 4))
    assert rc == 0
    nbytes = 64 * 8
    base = 1 << 40
    lin = (ctypes.c_void_p * 6)(*[base + i * nbytes for i in range(6)])
    lout = (ctypes.c_void_p * 6)(*[base + (6 + i) * nbytes for i in range(6)])
    en = (ctypes.c_void_p * 3)(*[base + (12 + i) * nbytes for i in range(3)])
    g = (ctypes.c_double * 12)()
    # valid pointers: passes the host checks, then fails for lack of bound fields
    assert B.lib().xfdtd_adjoint_step(h, lin, lout, en, g) == -5
    shifted = (ctypes.c_void_p * 6)(*[base + (5 + i) * nbytes + 8 for i in range(6)])  # overlaps lin[5]
    assert B.lib().xfdtd_adjoint_step(h, lin, shifted, en, g) == -1
    on_e = (ctypes.c_void_p * 6)(*[base + (6 + i) * nbytes for i in range(5)] + [base + 13 * nbytes])
    assert B.lib().xfdtd_adjoint_step(h, lin, on_e, en, g) == -1
    dup = (ctypes.c_void_p * 6)(*[base + (6 + i) * nbytes for i in range(5)] + [base + 6 * nbytes])
    assert B.lib().xfdtd_adjoint_step(h, lin, dup, en, g) == -1
    B.lib().xfdtd_destroy(h)


def test_error_messages_are_per_thread():
    """xfdtd_last_error reports the last failure of the calling thread: two
    threads failing with different errors at the same time each read their
    own message (ctypes releases the GIL around the calls)."""
    import threading

    barrier = threading.Barrier(2)
    seen = {}

    def worker(name, shape, dt):
        g = B.make_grid(shape)
        h = ctypes.c_void_p()
        c = B.dbl_array(O.yee_coeffs(), 12)
        for _ in range(200):
            barrier.wait()
            rc = B.lib().xfdtd_create(ctypes.byref(g), dt, c, B.XFDTD_F64, 0, ctypes.byref(h))
            barrier.wait()
            seen.setdefault(name, set()).add((rc, B.lib().xfdtd_last_error()))

    t1 = threading.Thread(target=worker, args=("grid", (0, 4, 4), 0.3))
    t2 = threading.Thread(target=worker, args=("dt", (4, 4, 4), -1.0))
    t1.start(), t2.start()
    t1.join(), t2.join()
    assert seen["grid"] == {(-1, b"invalid grid (sizes >= 1, spacings > 0)")}
    assert len(seen["dt"]) == 1 and b"dt" in next(iter(seen["dt"]))[1]


def test_empty_inputs():
    """Zero-length requests are valid no-ops that touch no pointer; negative
    lengths and empty batches are argument errors (no device work either)."""
    g = B.make_grid((4, 4, 4))
    c = B.dbl_array(O.yee_coeffs(), 12)
    assert B.lib().xfdtd_dispersion(ctypes.byref(g), 0.3, c, None, 0, None, None, None, None) == 0
    assert B.lib().xfdtd_dispersion(ctypes.byref(g), 0.3, c, None, -1, None, None, None, None) == -1
    h = ctypes.c_void_p()
    grids = (B.Grid * 1)(g)
    dts = (ctypes.c_double * 1)(0.3)
    assert B.lib().xfdtd_batch_create(grids, dts, c, 0, B.XFDTD_F32, 0, ctypes.byref(h)) == -1
    assert b"box count" in B.lib().xfdtd_last_error()


def test_batch_default_zsplit_fills_the_cus():
    """Untuned batches split z so that a small batch still has work for every
    CU (one 96^3 box: 24 tiles), but leave large boxes whole."""
    beta, delta = S.extended_beta_delta(9)
    c = O.coeffs_from(beta, delta)
    dt = 0.9 * O.cfl_dt(c)

    def zsplit(shapes):
        m = len(shapes)
        grids = (B.Grid * m)(*[B.make_grid(sh) for sh in shapes])
        dts = (ctypes.c_double * m)(*([dt] * m))
        cc = (ctypes.c_double * (12 * m))(*(list(c) * m))
        h = ctypes.c_void_p()
        assert B.lib().xfdtd_batch_create(grids, dts, cc, m, B.XFDTD_F32, 0, ctypes.byref(h)) == 0
        v = [ctypes.c_int() for _ in range(5)]
        assert B.lib().xfdtd_batch_get_config(h, *[ctypes.byref(x) for x in v]) == 0
        B.lib().xfdtd_batch_destroy(h)
        return v[0].value, v[1].value, v[2].value

    tx, ty, zs = zsplit([(96, 96, 96)])
    chunk = max(-(-96 // zs), 4)
    assert -(-96 // tx) * -(-96 // ty) * -(-96 // chunk) >= 256
    assert zsplit([(256, 256, 512)])[2] == 1


def test_batch_bind_rejects_overlap_before_device_work():
    c = O.yee_coeffs()
    grids = (B.Grid * 2)(B.make_grid((4, 4, 4)), B.make_grid((4, 4, 4)))
    dts = (ctypes.c_double * 2)(0.3, 0.3)
    cc = (ctypes.c_double * 24)(*(list(c) * 2))
    h = ctypes.c_void_p()
    assert B.lib().xfdtd_batch_create(grids, dts, cc, 2, B.XFDTD_F64, 0, ctypes.byref(h)) == 0
    base, nb = 1 << 40, 64 * 8
    f = (ctypes.c_void_p * 12)(*[base + i * nb for i in range(12)])
    s = (ctypes.c_void_p * 12)(*[base + (12 + i) * nb for i in range(12)])
    s_bad = (ctypes.c_void_p * 12)(*[base + (11 + i) * nb for i in range(12)])
    assert B.lib().xfdtd_batch_bind(h, f, s_bad, None) == -1
    f_mis = (ctypes.c_void_p * 12)(*[base + 4 + i * nb for i in range(12)])
    assert B.lib().xfdtd_batch_bind(h, f_mis, s, None) == -1
    B.lib().xfdtd_batch_destroy(h)


def test_stencil_family_builds_the_affine_problem():
    """Host-side marshalling of the minimiser's problem (no GPU call)."""
    from paper_1710_06829_amd.norm import NAMES
    fam = (pkg.Family({"dt": 0.5}).param(-0.1, 0.2, beta_xy=1, beta_yx=1)
           .param(-0.125, 0.125, delta_x=1, delta_y=0.5))
    p = fam.problem(dims=2, n=100, weight="axis", width=0.1, starts=3, max_iter=50)
    assert p.nparam == 2 and p.alpha_rule == 1 and p.dt_mode == 0
    assert p.base[NAMES.index("dt")] == 0.5
    assert p.map[NAMES.index("beta_yx") * 8 + 0] == 1.0 and p.map[NAMES.index("delta_y") * 8 + 1] == 0.5
    assert p.map[NAMES.index("delta_x") * 8 + 0] == 0.0
    assert (p.lo[0], p.hi[0], p.lo[1], p.hi[1]) == (-0.1, 0.2, -0.125, 0.125)
    assert p.weight == B.XFDTD_WEIGHT_AXIS and p.width == 0.1 and p.n == 100 and p.dims == 2
    fam2 = pkg.Family().param(0, 0.1, beta_xy=1).dt_fraction(0.2, 1.0)
    p2 = fam2.problem(dims=3, n=10, weight="unit", width=0.1, starts=2, max_iter=5)
    assert p2.dt_mode == 1 and p2.dt_param == 1
    with pytest.raises(ValueError):
        fam2.dt_fraction(0.1, 1.0)


def test_absurd_workspace_sizes_are_argument_errors():
    # no 64-bit overflow of the workspace size and no exception: a plain
    # XFDTD_EINVAL before any device call
    rc, h = _create(shape=(1024, 1024, 256))
    assert rc == 0
    L = B.lib()
    out = ctypes.c_uint64()
    try:
        for n, seg in [(1 << 62, 0), ((1 << 40) + 1, 0), (100, 1 << 50), (1 << 40, 1)]:
            rc = L.xfdtd_grad_workspace(h, n, seg, ctypes.byref(out))
            assert rc == -1, (n, seg, rc)
            assert L.xfdtd_last_error()
        assert L.xfdtd_grad_workspace(h, 200, 0, ctypes.byref(out)) == 0 and out.value > 0
    finally:
        L.xfdtd_destroy(h)


_ALLOC_CHILD = r"""
import ctypes, resource, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_1710_06829_amd import _binding as B
L = B.lib()
m = 1 << 20
grids = (B.Grid * m)()
for i in range(0, m, 4096):
    grids[i] = B.make_grid((4, 4, 4), (1, 1, 1))
for i in range(m):
    if i % 4096:
        ctypes.memmove(ctypes.byref(grids, i * ctypes.sizeof(B.Grid)), ctypes.byref(grids, 0),
                       ctypes.sizeof(B.Grid))
dts = np.full(m, 0.3)
coeffs = np.tile(np.array([1.0, 0, 0, 0] * 3), m)
out = ctypes.c_void_p()
# leave ~32 MB of address space: the batch's host vectors (~160 MB) cannot fit
used = int(open("/proc/self/statm").read().split()[0]) * resource.getpagesize()
resource.setrlimit(resource.RLIMIT_AS, (used + (32 << 20), resource.RLIM_INFINITY))
rc = L.xfdtd_batch_create(grids, dts.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          coeffs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m, B.XFDTD_F64, 1,
                          ctypes.byref(out))
print("rc", rc, L.xfdtd_last_error().decode())
"""


def test_host_allocation_failure_is_an_error_code_not_an_exception():
    # A failed host allocation inside an entry point (here the per-box vectors
    # of a 2^20-box batch under an address-space limit) must come back as
    # XFDTD_EINVAL with a message; a C++ exception crossing the C interface
    # would terminate the process instead.
    import subprocess
    import sys
    r = subprocess.run([sys.executable, "-c", _ALLOC_CHILD, ROOT], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "rc -1 out of host memory" in r.stdout, r.stdout + r.stderr[-2000:]


def test_stats_of_a_fresh_handle_and_argument_errors():
    """xfdtd_stats on a created, unbound handle: all counters zero, no timing
    (-1); reset with timing on needs no device; null arguments are errors."""
    rc, h = _create()
    assert rc == 0
    try:
        st = B.Stats()
        assert B.lib().xfdtd_get_stats(h, ctypes.byref(st)) == 0
        assert st.steps == 0 and st.run_calls == 0 and st.model_bytes == 0.0
        assert st.elapsed_ms == -1.0 and st.gcells_per_s == -1.0
        assert B.lib().xfdtd_reset_stats(h, 1) == 0
        assert B.lib().xfdtd_get_stats(h, ctypes.byref(st)) == 0 and st.elapsed_ms == -1.0
        assert B.lib().xfdtd_get_stats(h, None) == -1
        assert B.lib().xfdtd_get_stats(None, ctypes.byref(st)) == -1
        assert B.lib().xfdtd_reset_stats(None, 0) == -1
    finally:
        B.lib().xfdtd_destroy(h)


def test_log_prints_the_configuration_and_roctx_is_linked():
    """XFDTD_LOG=1: xfdtd_create prints its launch configuration to stderr (a
    child process, host only); the library links ROCm's roctx library for its
    ranges."""
    code = (
        "import ctypes, sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from paper_1710_06829_amd import _binding as B\n"
        "g = B.Grid(64, 48, 40, 1.0, 1.0, 1.0)\n"
        "c = (ctypes.c_double * 12)(*([1.0, 0, 0, 0] * 3))\n"
        "h = ctypes.c_void_p()\n"
        "assert B.lib().xfdtd_create(ctypes.byref(g), 0.5, c, 1, 0, ctypes.byref(h)) == 0\n"
        "B.lib().xfdtd_destroy(h)\n"
    )
    env = dict(os.environ, XFDTD_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "[xfdtd] create 64x48x40 FP32" in r.stderr, r.stderr
    r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, XFDTD_LOG="0"),
                       capture_output=True, text=True, timeout=300)
    assert "[xfdtd]" not in r.stderr
    d = subprocess.run(["readelf", "-d", B.LIB_PATH], capture_output=True, text=True)
    if d.returncode == 0:
        assert "librocprofiler-sdk-roctx" in d.stdout


def test_checked_run_needs_bound_fields():
    """xfdtd_run_checked on an unbound handle is a state error; done is 0."""
    rc, h = _create()
    assert rc == 0
    try:
        done = ctypes.c_int64(7)
        assert B.lib().xfdtd_run_checked(h, 10, 5, ctypes.byref(done)) == -5
        assert done.value == 0
    finally:
        B.lib().xfdtd_destroy(h)
