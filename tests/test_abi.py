"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point declared in include/gn.h, and rejects bad arguments before any
device work (those paths return without touching HIP)."""
import ctypes
import os
import re

import pytest

from paper_2009_11392_amd import _capi as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "gn.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\S.*?\b(gn_[a-z0-9_]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(C.LIB_PATH):
        pytest.fail("libgn.so is not built (run python -m paper_2009_11392_amd.build)")
    return C.lib()


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    assert set(syms) == set(C.EXPORTED), syms


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_status_strings_and_version(lib):
    assert lib.gn_status_string(0) == b"GN_OK"
    for code in range(1, 9):
        assert lib.gn_status_string(code).startswith(b"GN_ERR_")
    assert re.match(rb"\d+\.\d+\.\d+", lib.gn_version())


def _prob(**kw):
    base = dict(m=2000, n=1000, r=50, l=25, kind_x=0, kind_y=0, seed=1, mode=0, core_method=0,
                eps=1e-15, nu_x=0.0, nu_y=0.0)
    base.update(kw)
    return C.GnProblem(**base)


def _ws(lib, p, op, kc=0):
    out = ctypes.c_size_t(0)
    code = lib.gn_workspace_size(ctypes.byref(p), op, kc, ctypes.byref(out))
    return code, out.value


def test_workspace_sizes(lib):
    p = _prob()
    code, b = _ws(lib, p, C.GN_OP_SKETCH)
    assert code == 0 and b >= 8 * (50 * 1000 + 75 * 2000)
    code, b = _ws(lib, p, C.GN_OP_CORE)
    assert code == 0 and b >= 8 * 75 * 50
    assert _ws(lib, p, C.GN_OP_APPLY, 0)[0] == C.GN_ERR_SHAPE
    code, b = _ws(lib, p, C.GN_OP_BACKWARD)
    assert code == 0 and b >= 4 * 2000 * (50 + 75)
    code, b = _ws(lib, p, C.GN_OP_MATERIALIZE)
    assert code == 0 and b >= 8 * (2000 * 50 + 50 * 1000)
    assert _ws(lib, p, 99)[0] == C.GN_ERR_ARG
    # the power-method check: nv start vectors of length r
    assert _ws(lib, p, C.GN_OP_CHECK, 0)[0] == C.GN_ERR_ARG
    assert _ws(lib, p, C.GN_OP_CHECK, 17)[0] == C.GN_ERR_ARG
    code, b = _ws(lib, p, C.GN_OP_CHECK, 8)
    assert code == 0 and b >= 8 * 8 * 50
    # the SVD route adds the Jacobi vectors and rotations (two r x r) and Q (r+l) x r
    qr_bytes = _ws(lib, p, C.GN_OP_CORE)[1]
    for method in (C.GN_CORE_SVD, C.GN_CORE_LIFT_SVD, C.GN_CORE_LIFT_RRQR):
        code, b = _ws(lib, _prob(core_method=method), C.GN_OP_CORE)
        assert code == 0 and b >= qr_bytes + 8 * (2 * 50 * 50 + 75 * 50)
    assert _ws(lib, _prob(core_method=C.GN_CORE_LIFT_DIAG), C.GN_OP_CORE)[1] == qr_bytes


@pytest.mark.parametrize("kw,code", [
    (dict(r=0), C.GN_ERR_SHAPE), (dict(r=1001), C.GN_ERR_SHAPE), (dict(m=0), C.GN_ERR_SHAPE),
    (dict(mode=7), C.GN_ERR_ARG), (dict(kind_x=5), C.GN_ERR_ARG), (dict(kind_y=1), C.GN_ERR_ARG),
    (dict(eps=float("nan")), C.GN_ERR_ARG), (dict(core_method=5), C.GN_ERR_ARG),
    (dict(core_method=-1), C.GN_ERR_ARG), (dict(core_method=2, eps=0.0), C.GN_ERR_ARG),
    (dict(core_method=4, eps=-1.0), C.GN_ERR_ARG),
    (dict(r=3000, l=2000, m=9000, n=9000), C.GN_ERR_UNSUPPORTED),
    (dict(kind_x=1, n=1 << 18, m=10), C.GN_ERR_SHAPE),
    (dict(kind_x=1, n=1 << 18, m=1 << 18), C.GN_ERR_UNSUPPORTED),
])
def test_problem_validation(lib, kw, code):
    assert _ws(lib, _prob(**kw), C.GN_OP_SKETCH)[0] == code


def test_entry_points_reject_before_enqueue(lib):
    p = _prob()
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(1 << 20)                 # never dereferenced: rejected first
    # null A
    assert lib.gn_sketch(ctypes.byref(p), null, 1000, null, null, 0, null, 0, fake, 50, fake,
                         1000, null, null, fake, 1 << 30, null) == C.GN_ERR_ARG
    # lda < n
    assert lib.gn_sketch(ctypes.byref(p), fake, 999, null, null, 0, null, 0, fake, 50, fake,
                         1000, null, null, fake, 1 << 30, null) == C.GN_ERR_SHAPE
    # misaligned output
    assert lib.gn_sketch(ctypes.byref(p), fake, 1000, null, null, 0, null, 0,
                         ctypes.c_void_p((1 << 20) + 4), 50, fake, 1000, null, null, fake,
                         1 << 30, null) == C.GN_ERR_ALIGN
    # workspace too small
    assert lib.gn_sketch(ctypes.byref(p), fake, 1000, null, null, 0, null, 0, fake, 50, fake,
                         1000, null, null, fake, 16, null) == C.GN_ERR_WORKSPACE
    # BF16 mode needs scales
    pb = _prob(mode=2)
    assert lib.gn_sketch(ctypes.byref(pb), fake, 1000, null, null, 0, null, 0, fake, 50, fake,
                         1000, null, null, fake, 1 << 30, null) == C.GN_ERR_ARG
    # core output struct with a null member
    out = C.GnCoreOut(1 << 20, 0, 1 << 20, 1 << 20, 1 << 20, 1 << 20)
    assert lib.gn_core(ctypes.byref(p), fake, 50, null, 0, null, 0, ctypes.byref(out), fake,
                       1 << 30, null) == C.GN_ERR_ARG
    assert lib.gn_apply(ctypes.byref(p), 3, fake, 50, fake, 1000, ctypes.byref(out), fake, 1, 1,
                        fake, 1, fake, 1 << 30, null) == C.GN_ERR_ARG
    good = C.GnCoreOut(1 << 20, 1 << 20, 1 << 20, 1 << 20, 1 << 20, 1 << 20)
    # gn_core_check: every case fails a check before anything is enqueued
    def chk(prob=p, core=good, delta=0.0, nv=8, iters=4, ws_bytes=1 << 34):
        return lib.gn_core_check(ctypes.byref(prob), ctypes.byref(core), delta, nv, iters, null,
                                 fake, ws_bytes, null)
    assert chk(core=out) == C.GN_ERR_ARG                      # null status
    assert chk(nv=0) == C.GN_ERR_ARG and chk(nv=17) == C.GN_ERR_ARG
    assert chk(iters=0) == C.GN_ERR_ARG and chk(iters=65) == C.GN_ERR_ARG
    assert chk(prob=_prob(eps=0.0)) == C.GN_ERR_ARG            # no threshold at all
    assert chk(delta=float("inf")) == C.GN_ERR_ARG
    assert chk(ws_bytes=64) == C.GN_ERR_WORKSPACE
    # side 2 (materialize): ldo < n, then a workspace too small
    assert lib.gn_apply(ctypes.byref(p), 2, fake, 50, fake, 1000, ctypes.byref(good), null, 0, 0,
                        fake, 999, fake, 1 << 30, null) == C.GN_ERR_SHAPE
    assert lib.gn_apply(ctypes.byref(p), 2, fake, 50, fake, 1000, ctypes.byref(good), null, 0, 0,
                        fake, 1000, fake, 64, null) == C.GN_ERR_WORKSPACE
    # gn_backward: unsupported kinds / modes, missing operands, strides, workspace
    big = 1 << 34
    def back(prob, A=fake, lda=1000, G=fake, ldg=1000, AX=fake, ldax=50, ws_bytes=big, core=good):
        return lib.gn_backward(ctypes.byref(prob), A, lda, G, ldg, AX, ldax, fake, 1000,
                               ctypes.byref(core), fake, 1000, fake, ws_bytes, null)
    assert back(_prob(kind_x=1)) == C.GN_ERR_UNSUPPORTED
    assert back(_prob(mode=2)) == C.GN_ERR_UNSUPPORTED
    assert back(_prob(core_method=C.GN_CORE_SVD)) == C.GN_ERR_UNSUPPORTED   # QR cores only
    assert back(p, G=null) == C.GN_ERR_ARG
    assert back(p, A=null, AX=null) == C.GN_ERR_ARG
    nok = C.GnCoreOut(0, 1 << 20, 1 << 20, 1 << 20, 1 << 20, 1 << 20)   # k pointer null
    assert back(p, core=nok) == C.GN_ERR_ARG
    assert back(p, ldg=999) == C.GN_ERR_SHAPE
    assert back(p, ldax=49) == C.GN_ERR_SHAPE
    assert back(p, AX=null, lda=999) == C.GN_ERR_SHAPE
    assert back(p, ws_bytes=1 << 10) == C.GN_ERR_WORKSPACE
    assert lib.gn_residual(10, 10, 2, fake, 5, 0, null, fake, 2, fake, 10, fake, fake, 1 << 20,
                           null) == C.GN_ERR_SHAPE
    assert lib.gn_quantize_bf16_bs(10, 10, fake, 10, 2, fake, 10, fake, null) == C.GN_ERR_DTYPE
    assert lib.gn_generate_gaussian(1, 1, 0, 0, 4, 4, 5, 0, fake, 4, null) == C.GN_ERR_ARG
    assert lib.gn_srht_generate(1, 100, 200, fake, fake, fake, 1 << 20, null) == C.GN_ERR_SHAPE


def test_batch_validation_rejects_before_enqueue(lib):
    fake = 1 << 20
    core = C.GnCoreOut(fake, fake, fake, fake, fake, fake)

    def arr(**kw):
        base = dict(m=300, n=200, r=20, l=10, seed=1, eps=1e-7, A=fake, lda=200, AX=fake, ldax=20,
                    YtA=fake, ldya=200, core=core)
        base.update(kw)
        a = (C.GnBatchProblem * 2)()
        a[0] = C.GnBatchProblem(**base)
        a[1] = C.GnBatchProblem(**dict(base, m=base["m"] + 17))
        return a

    nb = ctypes.c_size_t(0)
    assert lib.gn_batch_workspace_size(arr(), 2, ctypes.byref(nb)) == C.GN_OK and nb.value > 0
    assert lib.gn_batch_workspace_size(arr(), 0, ctypes.byref(nb)) == C.GN_ERR_ARG
    assert lib.gn_batch_workspace_size(arr(r=201), 2, ctypes.byref(nb)) == C.GN_ERR_SHAPE
    assert lib.gn_batch_workspace_size(arr(lda=201), 2, ctypes.byref(nb)) == C.GN_ERR_ALIGN
    assert lib.gn_batch_workspace_size(arr(ldax=21), 2, ctypes.byref(nb)) == C.GN_ERR_ALIGN
    assert lib.gn_batch_workspace_size(arr(m=600, n=600, r=400, l=200, lda=600, ldya=600, ldax=400), 2,
                                       ctypes.byref(nb)) == C.GN_ERR_UNSUPPORTED
    assert lib.gn_batch_workspace_size(arr(A=0), 2, ctypes.byref(nb)) == C.GN_ERR_ARG
    plan = C.GnBatchPlan()
    # workspace too small / bad tile policy: rejected before any copy or launch
    assert lib.gn_batch_prepare(arr(), 2, None, ctypes.byref(plan), ctypes.c_void_p(fake), 64,
                                None) == C.GN_ERR_WORKSPACE
    bad = (ctypes.c_int32 * 4)(0, 1, 5, 1)
    assert lib.gn_batch_prepare(arr(), 2, bad, ctypes.byref(plan), ctypes.c_void_p(fake),
                                nb.value, None) == C.GN_ERR_ARG
    bad = (ctypes.c_int32 * 4)(0, 1, 3, 1)   # mixes 256- and 512-thread tiles
    assert lib.gn_batch_prepare(arr(), 2, bad, ctypes.byref(plan), ctypes.c_void_p(fake),
                                nb.value, None) == C.GN_ERR_ARG
    assert lib.gn_batch_solve(ctypes.byref(C.GnBatchPlan()), 3, ctypes.c_void_p(fake), 1 << 30,
                              None) == C.GN_ERR_ARG
    assert lib.gn_batch_solve(ctypes.byref(C.GnBatchPlan()), 0, ctypes.c_void_p(fake), 1 << 30,
                              None) == C.GN_ERR_ARG


def test_update_entry_points_reject_before_enqueue(lib):
    fake = ctypes.c_void_p(1 << 20)
    big = 1 << 34
    p = _prob()                                   # 2000 x 1000, r = 50, l = 25, FP64
    pn = _prob(r=60, l=30)
    # extend: r must grow, kinds / seeds must agree, BF16 unsupported, workspace
    assert lib.gn_sketch_extend(ctypes.byref(pn), ctypes.byref(p), fake, 1000, fake, 60, fake,
                                1000, fake, big, None) == C.GN_ERR_SHAPE
    assert lib.gn_sketch_extend(ctypes.byref(p), ctypes.byref(_prob(r=60, l=30, seed=2)), fake,
                                1000, fake, 60, fake, 1000, fake, big, None) == C.GN_ERR_ARG
    assert lib.gn_sketch_extend(ctypes.byref(_prob(mode=2)), ctypes.byref(_prob(mode=2, r=60)),
                                fake, 1000, fake, 60, fake, 1000, fake, big, None) == \
        C.GN_ERR_UNSUPPORTED
    assert lib.gn_sketch_extend(ctypes.byref(p), ctypes.byref(pn), fake, 1000, fake, 59, fake,
                                1000, fake, big, None) == C.GN_ERR_SHAPE
    assert lib.gn_sketch_extend(ctypes.byref(p), ctypes.byref(pn), fake, 1000, fake, 60, fake,
                                1000, fake, 64, None) == C.GN_ERR_WORKSPACE
    # append: axis, old size range, SRHT columns unsupported, ldb
    assert lib.gn_sketch_append(ctypes.byref(p), 2, 1500, fake, 1000, fake, 50, fake, 1000, fake,
                                big, None) == C.GN_ERR_ARG
    assert lib.gn_sketch_append(ctypes.byref(p), 0, 2000, fake, 1000, fake, 50, fake, 1000, fake,
                                big, None) == C.GN_ERR_SHAPE
    assert lib.gn_sketch_append(ctypes.byref(p), 0, 40, fake, 1000, fake, 50, fake, 1000, fake,
                                big, None) == C.GN_ERR_SHAPE
    assert lib.gn_sketch_append(ctypes.byref(_prob(kind_x=1)), 1, 900, fake, 100, fake, 50, fake,
                                1000, fake, big, None) == C.GN_ERR_UNSUPPORTED
    assert lib.gn_sketch_append(ctypes.byref(p), 1, 900, fake, 99, fake, 50, fake, 1000, fake,
                                big, None) == C.GN_ERR_SHAPE
    # update: strides, null E, workspace
    assert lib.gn_sketch_update(ctypes.byref(p), fake, 999, fake, 50, fake, 1000, fake, big,
                                None) == C.GN_ERR_SHAPE
    assert lib.gn_sketch_update(ctypes.byref(p), None, 1000, fake, 50, fake, 1000, fake, big,
                                None) == C.GN_ERR_ARG
    assert lib.gn_sketch_update(ctypes.byref(p), fake, 1000, fake, 50, fake, 1000, fake, 64,
                                None) == C.GN_ERR_WORKSPACE
