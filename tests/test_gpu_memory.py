"""Device memory of a handle against the host-side count of Eq. (2)'s model
(chase_workspace_bytes), measured as the drop in free device memory."""
import ctypes

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_15595_amd import _lib
    _lib.load()
    torch.cuda.init()
    # first handle of the process: the HIP context, code objects and the
    # rocBLAS/rocSOLVER libraries load here, outside the measured window
    for create in (_lib.load().chase_create, _lib.load().chase_create_real, _lib.load().chase_create_c64):
        h = ctypes.c_void_p()
        prm = _lib.default_params(nev=8, nex=4)
        assert create(256, ctypes.byref(prm), ctypes.byref(h)) == 0
        _lib.chase_destroy(h)
    return _lib


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("variant,prec", [(0, "fp64"), (0, "fp32"), (0, "bf16x3"), (1, "fp64"), (2, "fp64")])
def test_create_allocates_the_counted_bytes(L, variant, prec):
    """Every buffer is one hipMalloc rounded up to the allocator's page, and
    the HIP runtime may reserve memory of its own on the handle's first
    launches: the drop in free memory lies between the count and the count
    plus 256 MiB, and destroy returns it."""
    code = {"fp64": L.CHASE_FP64, "fp32": L.CHASE_FP32_MIXED, "bf16x3": L.CHASE_BF16X3_MIXED}[prec]
    N = 12001 if variant == 1 else 12000
    prm = L.default_params(nev=500, nex=100, precision=code)
    counted = L.chase_workspace_bytes(N, prm, variant)
    create = {0: L.load().chase_create, 1: L.load().chase_create_real, 2: L.load().chase_create_c64}[variant]
    before = _free()
    h = ctypes.c_void_p()
    assert create(N, ctypes.byref(prm), ctypes.byref(h)) == 0
    try:
        if variant == 1:   # the padded copy of H of an odd order is allocated by the first solve
            counted -= 8 * (N + 1) * (N + 1)
        used = before - _free()
    finally:
        L.chase_destroy(h)
    after = before - _free()
    print(f"\nvariant {variant} {prec}: counted {counted / 2**20:.1f} MiB, used {used / 2**20:.1f} MiB")
    assert counted <= used <= counted + (256 << 20)
    assert abs(after) <= 64 << 20
