"""The library's plain copy kernel (the bandwidth reference of the roofline):
byte-exact for sizes with a partial last work group and a tail that is not a
whole 16-byte vector, and it leaves the bytes past the copied range alone."""

import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2008_01473_amd import runtime  # noqa: E402  (raises if liblbm.so is missing)


@pytest.mark.parametrize("nbytes", [0, 5, 16, 4096, 4096 + 7, 16 * 256 * 3 + 16 * 5 + 9, (64 << 20) + 48])
def test_copy_kernel_is_byte_exact(nbytes):
    g = torch.Generator(device="cpu").manual_seed(nbytes)
    n_alloc = nbytes + 64
    src = torch.randint(0, 256, (n_alloc,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(n_alloc, dtype=torch.uint8, device="cuda")
    print(f"case copy {nbytes} bytes", flush=True)
    runtime.copy_kernel(dst, src, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes].cpu(), src[:nbytes].cpu())
    assert int(dst[nbytes:].count_nonzero()) == 0
