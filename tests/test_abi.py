"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments before any HIP call (no GPU needed: no compute call is made).

Every call below either fails validation or has n == 0, so none reaches a
kernel launch: the stand-in addresses are never dereferenced."""
import ctypes

import pytest

from paper_1807_08084_amd import _lib as L

FAKE = 0x10000          # 16-byte aligned stand-in device addresses; never dereferenced
FAKE2 = 0x20000000
FAKE3 = 0x40000000


@pytest.fixture(scope="module")
def lib():
    return L.lib()


def test_exports_every_declared_symbol(lib):
    names = L.declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_recommended_pitch(lib):
    assert lib.polsar_recommended_pitch(L.F32, 1 << 24) == (1 << 24) + 8192
    assert lib.polsar_recommended_pitch(L.F64, 1 << 24) == (1 << 24) + 4096
    assert lib.polsar_recommended_pitch(L.F32, 1) == 16384 + 8192
    assert lib.polsar_recommended_pitch(L.F32, 0) == 8192
    assert lib.polsar_recommended_pitch(2, 10) == -1 and lib.polsar_recommended_pitch(L.F32, -1) == -1
    for n in (1, 1000, 12345, 1 << 20):
        p = lib.polsar_recommended_pitch(L.F32, n)
        assert p >= n and (p * 4) % (64 << 10) == 32 << 10


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.status_string(code) != "unknown status"
    assert L.status_string(7) == "unknown status"


def inv_det(lib, dtype=L.F32, method=L.ADJUGATE, prec=L.COMPENSATED, n=1024, z=FAKE, zp=1024,
            inv=FAKE2, ip=1024, det=FAKE3, status=None, counters=None):
    return lib.polsar_inv_det(dtype, method, prec, n, z, zp, inv, ip, det, status, counters, None)


def test_inv_det_argument_errors(lib):
    assert inv_det(lib, n=0) == L.OK                       # empty batch: no launch
    assert inv_det(lib, z=None) == L.E_ARG
    assert inv_det(lib, n=-1) == L.E_ARG
    assert inv_det(lib, zp=1000) == L.E_ARG                # pitch < n
    assert inv_det(lib, ip=1000) == L.E_ARG
    assert inv_det(lib, dtype=2) == L.E_ARG
    assert inv_det(lib, method=2) == L.E_ARG
    assert inv_det(lib, prec=3) == L.E_ARG
    assert inv_det(lib, dtype=L.F64, prec=L.WIDE) == L.E_UNSUPPORTED
    assert inv_det(lib, dtype=L.F64, method=L.CHOLESKY, prec=L.COMPENSATED) == L.E_UNSUPPORTED
    assert inv_det(lib, z=FAKE + 2) == L.E_ALIGN           # not aligned to 4 bytes
    assert inv_det(lib, dtype=L.F64, z=FAKE + 4) == L.E_ALIGN
    assert inv_det(lib, det=FAKE3 + 1) == L.E_ALIGN
    assert inv_det(lib, inv=None, det=None) == L.E_ARG     # nothing to compute
    assert inv_det(lib, n=0, inv=FAKE + 64) == L.OK        # n == 0: no overlap to check


def test_inv_det_aliasing(lib):
    assert inv_det(lib, inv=FAKE, ip=1024, n=0) == L.OK
    assert inv_det(lib, inv=FAKE + 4096) == L.E_ALIAS       # overlaps z, not in place
    assert inv_det(lib, inv=FAKE, ip=2048, zp=1024) == L.E_ALIAS  # same base, other pitch
    assert inv_det(lib, det=FAKE + 4 * 9000) == L.E_ALIAS   # det inside z's span
    assert inv_det(lib, status=FAKE3 + 100) == L.E_ALIAS    # status inside det


def test_wishart_argument_errors(lib):
    def call(dtype=L.F32, mode=L.FWD, n=100, s=FAKE, sp=100, z=FAKE2, zp=100, N=4.0, loss=FAKE3,
             ell=None, gl=None, grad=None, gp=100, ws=FAKE3 + 4096, wsb=1 << 20):
        return lib.polsar_wishart_loglik(dtype, mode, n, s, sp, z, zp, N, loss, ell, gl, grad, gp, ws, wsb,
                                         None, None)
    assert lib.polsar_wishart_workspace_bytes(L.F32, 100) == ((100 + 63) // 64) * 8
    assert call(mode=0) == L.E_ARG
    assert call(N=0.0) == L.E_ARG
    assert call(s=None) == L.E_ARG
    assert call(loss=None) == L.E_ARG
    assert call(ws=None) == L.E_WORKSPACE
    assert call(wsb=0) == L.E_WORKSPACE
    assert call(mode=L.BWD, grad=None) == L.E_ARG
    assert call(mode=L.BWD, grad=FAKE + 64) == L.E_ALIAS
    assert call(loss=FAKE3 + 4) == L.E_ALIGN
    assert call(mode=L.BWD, n=0, grad=FAKE3) == L.OK


def test_launch_table(lib):
    c = L.Launch()
    assert lib.polsar_get_launch(0, L.F32, L.ADJUGATE, L.COMPENSATED, ctypes.byref(c)) == L.OK
    assert c.block in (64, 128, 256) and c.unroll in (1, 2, 4)
    bad = L.Launch(block=96, unroll=1, grid_per_cu=0, nontemporal=1, vector_bytes=16)
    assert lib.polsar_set_launch(0, L.F32, L.ADJUGATE, L.PLAIN, ctypes.byref(bad)) == L.E_ARG
    bad = L.Launch(block=128, unroll=4, grid_per_cu=0, nontemporal=1, vector_bytes=16)
    assert lib.polsar_set_launch(1, L.F32, 0, 0, ctypes.byref(bad)) == L.E_ARG   # wishart: unroll <= 2
    bad = L.Launch(block=128, unroll=1, grid_per_cu=0, nontemporal=1, vector_bytes=4)
    assert lib.polsar_set_launch(0, L.F32, L.ADJUGATE, L.PLAIN, ctypes.byref(bad)) == L.E_ARG
    bad = L.Launch(block=128, unroll=1, grid_per_cu=0, nontemporal=1, vector_bytes=16, blocks_per_cu=-1)
    assert lib.polsar_set_launch(0, L.F32, L.ADJUGATE, L.PLAIN, ctypes.byref(bad)) == L.E_ARG
    bad = L.Launch(block=128, unroll=2, grid_per_cu=8, nontemporal=1, vector_bytes=16, blocks_per_cu=0)
    assert lib.polsar_set_launch(3, L.F32, L.ADJUGATE, L.PLAIN, ctypes.byref(bad)) == L.E_ARG    # batch: unroll 1
    keep = L.Launch()
    assert lib.polsar_get_launch(3, L.F32, L.ADJUGATE, L.PLAIN, ctypes.byref(keep)) == L.OK
    tile = L.Launch(block=128, unroll=1, grid_per_cu=0, nontemporal=1, vector_bytes=16, blocks_per_cu=0)
    assert lib.polsar_set_launch(3, L.F32, L.ADJUGATE, L.PLAIN, ctypes.byref(tile)) == L.OK  # batch: one block per tile
    assert lib.polsar_set_launch(3, L.F32, L.ADJUGATE, L.PLAIN, ctypes.byref(keep)) == L.OK
    good = L.Launch(block=128, unroll=2, grid_per_cu=4, nontemporal=0, vector_bytes=8, blocks_per_cu=4)
    assert lib.polsar_set_launch(0, L.F64, L.CHOLESKY, L.PLAIN, ctypes.byref(good)) == L.OK
    got = L.Launch()
    lib.polsar_get_launch(0, L.F64, L.CHOLESKY, L.PLAIN, ctypes.byref(got))
    assert got.as_dict() == good.as_dict()
    # op 4, the copy probe: one tile per block, unroll 1
    assert lib.polsar_get_launch(4, L.F32, 0, 0, ctypes.byref(got)) == L.OK
    assert got.unroll == 1 and got.grid_per_cu == 0
    assert lib.polsar_set_launch(4, L.F32, 0, 0, ctypes.byref(good)) == L.E_ARG
    # op 5, the Wishart kernel on small images, op 6, the inverse on large
    # images, and the op a call of n pixels uses; op 7 does not exist
    assert lib.polsar_get_launch(5, L.F32, 0, 0, ctypes.byref(got)) == L.OK
    assert lib.polsar_get_launch(6, L.F32, L.ADJUGATE, L.COMPENSATED, ctypes.byref(got)) == L.OK
    assert lib.polsar_get_launch(7, L.F32, 0, 0, ctypes.byref(got)) == L.E_ARG
    assert lib.polsar_inv_det_launch_op(8192 * 8192) == 6 and lib.polsar_inv_det_launch_op(4096 * 4096) == 0
    assert lib.polsar_inv_det_launch_op((1 << 25) - 1) == 0 and lib.polsar_inv_det_launch_op(1 << 25) == 6
    assert lib.polsar_wishart_launch_op(2048 * 2048) == 5 and lib.polsar_wishart_launch_op(4096 * 4096) == 1
    assert lib.polsar_wishart_launch_op((1 << 23) - 1) == 5 and lib.polsar_wishart_launch_op(1 << 23) == 1


def test_batch_and_copy_argument_errors(lib):
    h = ctypes.c_void_p()
    arr = (L.Image * 1)()
    assert lib.polsar_batch_create(arr, 1, L.F32, L.ADJUGATE, L.COMPENSATED, 1, None, None, 0, ctypes.byref(h)) == L.E_ARG
    assert lib.polsar_batch_create(arr, 0, L.F32, L.ADJUGATE, L.COMPENSATED, 1, None, None, 0, ctypes.byref(h)) == L.E_ARG
    arr[0].n, arr[0].z, arr[0].z_pitch, arr[0].det = 16, FAKE, 16, FAKE2
    assert lib.polsar_batch_create(arr, 1, L.F32, L.ADJUGATE, L.COMPENSATED, 8, None, None, 0, ctypes.byref(h)) == L.E_ARG
    assert lib.polsar_batch_create(arr, 1, L.F64, L.ADJUGATE, L.WIDE, 1, None, None, 0, ctypes.byref(h)) == L.E_UNSUPPORTED
    assert lib.polsar_batch_create(arr, 1, L.F32, L.ADJUGATE, L.PLAIN, 2, None, None, 0, ctypes.byref(h)) == L.E_ARG  # no sigma
    ok = (L.Image * 1)()
    ok[0].n, ok[0].z, ok[0].z_pitch = 64, FAKE, 64
    ok[0].inv, ok[0].inv_pitch, ok[0].det = FAKE + 256, 64, FAKE3   # inverse planes inside z's span
    assert lib.polsar_batch_create(ok, 1, L.F32, L.ADJUGATE, L.COMPENSATED, 1, None, None, 0, ctypes.byref(h)) == L.E_ALIAS
    ok[0].inv, ok[0].det = FAKE2, FAKE2 + 1024                        # det inside the inverse planes
    assert lib.polsar_batch_create(ok, 1, L.F32, L.ADJUGATE, L.COMPENSATED, 1, None, None, 0, ctypes.byref(h)) == L.E_ALIAS
    # one grid runs all images at once: an output of one image may not overlap
    # another image's input or output (inputs may be shared)
    two = (L.Image * 2)()
    for i in range(2):
        two[i].n, two[i].z, two[i].z_pitch = 64, FAKE, 64                   # both read the same z
        two[i].inv, two[i].inv_pitch, two[i].det = FAKE2 + 4096 * i, 64, FAKE3 + 1024 * i
    two[1].inv = FAKE2 + 256                                              # image 1's inverse inside image 0's
    assert lib.polsar_batch_create(two, 2, L.F32, L.ADJUGATE, L.COMPENSATED, 1, None, None, 0, ctypes.byref(h)) == L.E_ALIAS
    two[1].inv, two[1].det = FAKE2 + 4096, FAKE + 128                      # image 1's det inside image 0's z
    assert lib.polsar_batch_create(two, 2, L.F32, L.ADJUGATE, L.COMPENSATED, 1, None, None, 0, ctypes.byref(h)) == L.E_ALIAS
    two[1].det = FAKE3                                                     # the two det planes coincide
    assert lib.polsar_batch_create(two, 2, L.F32, L.ADJUGATE, L.COMPENSATED, 1, None, None, 0, ctypes.byref(h)) == L.E_ALIAS
    assert lib.polsar_batch_run(None, None) == L.E_ARG
    assert lib.polsar_batch_tiles(None) == -1
    assert lib.polsar_stream_copy(L.F32, 100, FAKE, 100, 5, FAKE2, 100, 10, None) == L.E_UNSUPPORTED
    assert lib.polsar_stream_copy(L.F32, 100, FAKE, 100, 9, FAKE + 64, 100, 10, None) == L.E_ALIAS
    assert lib.polsar_stream_copy(L.F32, 0, FAKE, 100, 9, FAKE2, 100, 10, None) == L.OK


def test_multilook_blockdiag_streamer_argument_errors(lib):
    ml = lib.polsar_multilook_inv_det
    assert ml(L.F32, L.ADJUGATE, L.COMPENSATED, 100, 0, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ARG
    assert ml(L.F32, L.ADJUGATE, L.COMPENSATED, 100, 4, FAKE, 99, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ARG
    assert ml(L.F64, L.ADJUGATE, L.WIDE, 100, 4, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_UNSUPPORTED
    assert ml(L.F32, L.ADJUGATE, L.COMPENSATED, 100, 4, FAKE, 100, None, 0, FAKE + 400, 100, FAKE3, None, None, None) == L.E_ALIAS
    assert ml(L.F32, L.ADJUGATE, L.COMPENSATED, 100, 4, FAKE, 100, None, 0, None, 0, None, None, None, None) == L.E_ARG
    assert ml(L.F32, L.ADJUGATE, L.COMPENSATED, 0, 4, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.OK
    bd = lib.polsar_blockdiag_inv_det
    assert bd(L.F32, L.ADJUGATE, L.COMPENSATED, 100, 0, FAKE, 100, FAKE2, 100, FAKE3, None, 0, None, None, None) == L.E_ARG
    assert bd(L.F32, L.ADJUGATE, L.COMPENSATED, 100, 2, FAKE, 100, FAKE + 800, 100, FAKE3, None, 0, None, None, None) == L.E_ALIAS
    assert bd(L.F32, L.ADJUGATE, L.COMPENSATED, 0, 2, FAKE, 100, FAKE, 100, FAKE3, None, 0, None, None, None) == L.OK
    h = ctypes.c_void_p()
    assert lib.polsar_streamer_create(L.F32, L.ADJUGATE, L.COMPENSATED, 0, ctypes.byref(h)) == L.E_ARG
    assert lib.polsar_streamer_create(L.F64, L.ADJUGATE, L.WIDE, 1024, ctypes.byref(h)) == L.E_UNSUPPORTED
    assert lib.polsar_streamer_run(None, 10, FAKE, 10, FAKE2, 10, FAKE3, None, None) == L.E_ARG


def test_boxcar_argument_errors(lib):
    """Every rejection happens before any launch (fake pointers)."""
    bx = lib.polsar_boxcar_inv_det
    ok = (L.F32, L.ADJUGATE, L.COMPENSATED)
    # 10 x 10 image: planes of 100
    assert bx(*ok, 10, 10, 4, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ARG   # radius > 3
    assert bx(*ok, 10, 10, -1, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ARG
    assert bx(*ok, -1, 10, 1, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ARG
    assert bx(*ok, 1 << 25, 1, 1, FAKE, 1 << 25, None, 0, FAKE2, 1 << 25, FAKE3, None, None, None) == L.E_ARG
    assert bx(*ok, 1 << 17, 1 << 17, 1, FAKE, 1 << 34, None, 0, FAKE2, 1 << 34, FAKE3, None, None, None) == L.E_ARG
    assert bx(*ok, 10, 10, 1, FAKE, 99, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ARG       # pitch < n
    assert bx(*ok, 10, 10, 1, None, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ARG      # null s
    assert bx(L.F64, L.ADJUGATE, L.WIDE, 10, 10, 1, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None,
              None) == L.E_UNSUPPORTED
    assert bx(*ok, 10, 10, 1, FAKE + 2, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.E_ALIGN
    assert bx(*ok, 10, 10, 1, FAKE, 100, None, 0, FAKE + 800, 100, FAKE3, None, None, None) == L.E_ALIAS  # inv in s
    assert bx(*ok, 10, 10, 1, FAKE, 100, FAKE2, 100, FAKE2 + 400, 100, FAKE3, None, None, None) == L.E_ALIAS
    assert bx(*ok, 10, 10, 1, FAKE, 100, None, 0, None, 0, None, None, None, None) == L.E_ARG       # no output
    assert bx(*ok, 0, 10, 1, FAKE, 100, None, 0, FAKE2, 100, FAKE3, None, None, None) == L.OK        # empty


def test_nlm_argument_errors(lib):
    nl = lib.polsar_nlm_wishart
    args = lambda dt, dist, H, W, r, N=4.0, h=16.0: nl(dt, dist, H, W, r, N, h, FAKE, H * W, FAKE2, H * W,  # noqa: E731
                                                       FAKE3, H * W, None, None)
    assert args(L.F32, 0, 10, 10, 17) == L.E_ARG                  # radius > 16
    assert args(L.F32, 2, 10, 10, 3) == L.E_ARG                   # unknown distance
    assert args(L.F32, 0, 10, 10, 3, N=0.0) == L.E_ARG
    assert args(L.F32, 0, 10, 10, 3, h=0.0) == L.E_ARG
    assert args(L.F32, 0, 4 * 65535 + 1, 1, 3) == L.E_ARG         # grid rows
    assert args(L.F64, 0, 4 * 65535 + 1, 1, 3) == L.E_ARG
    assert args(L.F32, 0, 10, (1 << 20) + 1, 3) == L.E_ARG
    assert nl(L.F32, 0, 10, 10, 3, 4.0, 16.0, FAKE, 100, FAKE2, 100, FAKE + 400, 100, None, None) == L.E_ALIAS
    assert args(L.F32, 0, 0, 10, 3) == L.OK                       # empty


def test_wishart_noalloc_rejects_sizes_beyond_its_scratch(lib):
    """2^20 + 1 tiles at the default launches (FP64: 128 pixels per tile;
    FP32 with 16-byte aligned planes: 1024): one more than the fixed scratch
    holds.  Rejected before any HIP call; nothing is launched."""
    for dtype, n in ((L.F64, (1 << 27) + 128), (L.F32, (1 << 30) + 1024)):
        rc = lib.polsar_wishart_loglik_noalloc(dtype, L.FWD, n, FAKE, n, FAKE2, n, 4.0, FAKE3, None, None, None, 0,
                                               None, None)
        assert rc == L.E_WORKSPACE
    assert lib.polsar_wishart_loglik_noalloc(L.F32, 0, 100, FAKE, 100, FAKE2, 100, 4.0, FAKE3, None, None, None,
                                             0, None, None) == L.E_ARG
    assert lib.polsar_wishart_loglik_noalloc(L.F32, L.FWD, 100, FAKE, 100, FAKE2, 100, 4.0, None, None, None,
                                             None, 0, None, None) == L.E_ARG
