"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function include/daba.h declares, the workspace size is
computed on the host, and invalid problems are rejected before any device
work."""

import ctypes as C
import subprocess

import numpy as np
import pytest

from synth import make_problem

B = pytest.importorskip("paper_2305_07026_amd.binding")


def _problem(prob, **over):
    keep = dict(cam=np.ascontiguousarray(prob["obs_camera"], np.int32),
                lm=np.ascontiguousarray(prob["obs_landmark"], np.int32),
                uv=np.ascontiguousarray(prob["obs_uv"], np.float64),
                cams=np.ascontiguousarray(prob["cameras"], np.float64),
                lms=np.ascontiguousarray(prob["landmarks"], np.float64))
    keep.update(over)
    P = C.POINTER
    st = B.DabaProblem(prob["n_cameras"], prob["n_landmarks"], keep["cam"].size,
                       keep["cam"].ctypes.data_as(P(C.c_int32)), keep["lm"].ctypes.data_as(P(C.c_int32)),
                       keep["uv"].ctypes.data_as(P(C.c_double)), keep["cams"].ctypes.data_as(P(C.c_double)),
                       keep["lms"].ctypes.data_as(P(C.c_double)), over.get("S", 4), None, None, 512.0)
    return st, keep


def _opts(**kw):
    d = dict(loss=1, loss_delta=1.0, xi=1e-9, eta=0.5, accelerate=1, inner_steps=1, precision=0, debug_flags=0)
    d.update(kw)
    return B.DabaOptions(**d)


@pytest.fixture(scope="module")
def prob():
    return make_problem("cam50-lm5k", n_cameras=12, n_landmarks=300, seed=21)


def test_exports_every_declared_function():
    names = B.header_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(B.lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_workspace_bytes_on_host(prob):
    st, _keep = _problem(prob)
    n64 = B.lib.daba_workspace_bytes(C.byref(st), C.byref(_opts()))
    n32 = B.lib.daba_workspace_bytes(C.byref(st), C.byref(_opts(precision=1)))
    assert n64 > 0 and n32 > n64  # the mixed form keeps FP32 copies besides the FP64 state
    big = make_problem("cam50-lm5k", n_cameras=12, n_landmarks=900, seed=21)
    st2, _k2 = _problem(big)
    assert B.lib.daba_workspace_bytes(C.byref(st2), C.byref(_opts())) > n64
    assert B.lib.daba_workspace_bytes(C.byref(st), C.byref(_opts(eta=0.0))) == 0


@pytest.mark.parametrize("case", ["bad_index", "nan_uv", "not_rotation", "bad_partitions", "bad_xi",
                                  "degenerate", "null_workspace"])
def test_create_rejects_before_device_work(prob, case):
    over, opts, ws = {}, _opts(), C.c_void_p(4096)
    if case == "bad_index":
        cam = np.ascontiguousarray(prob["obs_camera"], np.int32).copy()
        cam[3] = prob["n_cameras"]
        over["cam"] = cam
    elif case == "nan_uv":
        uv = prob["obs_uv"].copy()
        uv[5, 1] = np.nan
        over["uv"] = uv
    elif case == "not_rotation":
        cams = prob["cameras"].copy()
        cams[2, :9] *= 1.01
        over["cams"] = cams
    elif case == "bad_partitions":
        over["S"] = 65
    elif case == "bad_xi":
        opts = _opts(xi=0.0)
    elif case == "degenerate":
        lms = prob["landmarks"].copy()
        j = prob["obs_landmark"][0]
        lms[j] = prob["cameras"][prob["obs_camera"][0], 9:12]
        over["lms"] = lms
    elif case == "null_workspace":
        ws = None
    st, _keep = _problem(prob, **over)
    h = C.c_void_p()
    rc = B.lib.daba_create(C.byref(st), C.byref(opts), ws, 1 << 40, None, C.byref(h))
    expect = -5 if case == "degenerate" else -1
    assert rc == expect, (rc, B.lib.daba_last_error(None))
    assert not h.value
    assert len(B.lib.daba_last_error(None)) > 0


def test_stream_copy_rejects_bad_arguments_before_device_work():
    # every case fails its argument check before any HIP call
    a, b = 4096, 8192  # stand-in addresses, never dereferenced
    assert B.lib.daba_stream_copy(None, b, 64, 16, None) == -1
    assert B.lib.daba_stream_copy(a, None, 64, 16, None) == -1
    assert B.lib.daba_stream_copy(a, b, 65, 16, None) == -1  # not a multiple of 16
    assert B.lib.daba_stream_copy(a + 8, b, 64, 16, None) == -1  # misaligned
    assert B.lib.daba_stream_copy(a, b, 64, 0, None) == -1
    assert B.lib.daba_stream_copy(a, b, 0, 16, None) == B.DABA_OK  # nothing to copy


def _part_args(prob, **over):
    import ctypes as C
    import numpy as np
    keep = dict(cam=np.ascontiguousarray(prob["obs_camera"], np.int32),
                lm=np.ascontiguousarray(prob["obs_landmark"], np.int32),
                uv=np.ascontiguousarray(prob["obs_uv"], np.float64),
                cams=np.ascontiguousarray(over.pop("cameras", prob["cameras"]), np.float64),
                lms=np.ascontiguousarray(over.pop("landmarks", prob["landmarks"]), np.float64))
    P_ = C.POINTER
    pr = B.DabaProblem(prob["n_cameras"], prob["n_landmarks"], prob["n_obs"],
                       keep["cam"].ctypes.data_as(P_(C.c_int32)), keep["lm"].ctypes.data_as(P_(C.c_int32)),
                       keep["uv"].ctypes.data_as(P_(C.c_double)), keep["cams"].ctypes.data_as(P_(C.c_double)),
                       keep["lms"].ctypes.data_as(P_(C.c_double)), over.pop("n_partitions", 3), None, None, 512.0)
    opt = dict(loss=1, loss_delta=1.0, xi=1e-9, eta=0.5, accelerate=1, inner_steps=1, precision=0, debug_flags=0)
    opt.update(over)
    return keep, pr, B.DabaOptions(**opt)


def test_part_workspace_bytes_on_host(prob):
    import ctypes as C
    keep, pr, opt = _part_args(prob)
    n = B.lib.daba_part_workspace_bytes(C.byref(pr), C.byref(opt))
    # at least the per-observation camera-landmark Hessian blocks (27 doubles each)
    assert n >= 27 * 8 * prob["n_obs"]
    for bad in (dict(precision=1), dict(inner_steps=0), dict(xi=0.0), dict(n_partitions=65)):
        keep, pr, opt = _part_args(prob, **bad)
        assert B.lib.daba_part_workspace_bytes(C.byref(pr), C.byref(opt)) == 0, bad


@pytest.mark.parametrize("case", ["fp32", "inner0", "eta", "not_rotation", "degenerate", "null_ws"])
def test_part_create_rejects_before_device_work(prob, case):
    import ctypes as C
    import numpy as np
    over = {"fp32": dict(precision=1), "inner0": dict(inner_steps=0), "eta": dict(eta=1.5), "null_ws": {}}.get(case, {})
    if case == "not_rotation":
        c = prob["cameras"].copy()
        c[0, :9] *= 2.0
        over = dict(cameras=c)
    if case == "degenerate":
        lms = prob["landmarks"].copy()
        lms[prob["obs_landmark"][0]] = prob["cameras"][prob["obs_camera"][0], 9:12]
        over = dict(landmarks=lms)
    keep, pr, opt = _part_args(prob, **over)
    h = C.c_void_p()
    rc = B.lib.daba_part_create(C.byref(pr), C.byref(opt), None, 0, None, C.byref(h))
    assert rc == (-5 if case == "degenerate" else -1), (case, rc, B.lib.daba_part_last_error(None))
    assert not h.value
    assert B.lib.daba_part_last_error(None)


def test_part_rejects_a_partition_beyond_the_camera_limit():
    import ctypes as C
    big = make_problem("cam50-lm5k", n_cameras=2100, n_landmarks=200, seed=3)
    keep, pr, opt = _part_args(big, n_partitions=1)
    assert B.lib.daba_part_workspace_bytes(C.byref(pr), C.byref(opt)) == 0
    h = C.c_void_p()
    assert B.lib.daba_part_create(C.byref(pr), C.byref(opt), None, 0, None, C.byref(h)) == -1
    assert b"at most" in B.lib.daba_part_last_error(None)
    keep, pr, opt = _part_args(big, n_partitions=2)  # 1,050 cameras each: accepted
    assert B.lib.daba_part_workspace_bytes(C.byref(pr), C.byref(opt)) > 0


def test_size_limits_on_host():
    """The largest problem the packed observation words allow (cameras below
    2^24, landmarks below 2^26, 64 partitions) is sized; one more camera or
    landmark is rejected before anything is read, and so is a partition
    count above 64.  No observations, so that the limits stay cheap."""
    P = C.POINTER
    cams = np.tile(np.r_[np.eye(3).ravel(), 0.0, 0.0, 10.0, 500.0, 0.0, 0.0], (1, 1))
    lms = np.zeros((1, 3))
    empty_i, empty_d = np.zeros(1, np.int32), np.zeros(2)

    def sized(M, N, S):
        st = B.DabaProblem(M, N, 0, empty_i.ctypes.data_as(P(C.c_int32)), empty_i.ctypes.data_as(P(C.c_int32)),
                           empty_d.ctypes.data_as(P(C.c_double)), cams.ctypes.data_as(P(C.c_double)),
                           lms.ctypes.data_as(P(C.c_double)), S, None, None, 512.0)
        return B.lib.daba_workspace_bytes(C.byref(st), C.byref(_opts()))

    assert sized((1 << 24) - 1, 1, 64) > 0
    assert sized(1 << 24, 1, 64) == 0
    assert sized(1, 1 << 26, 1) == 0
    assert sized(1, 1, 65) == 0
    assert sized(1, 1, 0) == 0
