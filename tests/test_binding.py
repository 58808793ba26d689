"""The Python binding's convenience wrappers without a GPU: element types that
the entry points have no kernel for are refused with TypeError before any
device pointer reaches the library (a float16 or bfloat16 buffer read as FP32
would be read out of bounds), and host tensors are refused as well."""
import pytest
import torch

import paper_2201_03611_amd as rise


def t(*shape, dtype=torch.float32):
    return torch.zeros(*shape, dtype=dtype)


@pytest.mark.parametrize("dtype", [torch.bfloat16, torch.float16, torch.float64])
def test_gemm_backward_refuses_non_fp32(dtype):
    with pytest.raises(TypeError):
        rise.gemm_backward(t(8, 8), t(8, 8, dtype=dtype), t(8, 8))
    with pytest.raises(TypeError):
        rise.gemm_backward(t(8, 8, dtype=dtype), t(8, 8), t(8, 8))


@pytest.mark.parametrize("dtype", [torch.float16, torch.float64, torch.int32])
def test_wrappers_refuse_other_types(dtype):
    x = t(16, 16, dtype=dtype)
    with pytest.raises(TypeError):
        rise.gemm(x, t(16, 16))
    with pytest.raises(TypeError):
        rise.gemv(x, t(16))
    with pytest.raises(TypeError):
        rise.gemv(t(16, 16), t(16, dtype=dtype))
    with pytest.raises(TypeError):
        rise.stencil2d(x, t(3, 3))
    with pytest.raises(TypeError):
        rise.stencil2d_iterate(x, t(3, 3), 2)
    with pytest.raises(TypeError):
        rise.iterate_sum(x.reshape(-1), 2, 8)
    with pytest.raises(TypeError):
        rise.stencil2d_backward(x, t(16, 16), t(3, 3))
    with pytest.raises(TypeError):
        rise.conv2d(t(1, 4, 4, 32, dtype=dtype), t(32, 32, 3, 3))
    with pytest.raises(TypeError):
        rise.conv2d_backward(t(1, 4, 4, 32, dtype=dtype), t(1, 4, 4, 32, dtype=torch.bfloat16),
                             t(32, 32, 3, 3))


def test_host_tensors_are_refused():
    with pytest.raises(ValueError, match="device tensors"):
        rise.gemm(t(16, 16), t(16, 16))
    with pytest.raises(ValueError, match="device tensors"):
        rise.stencil2d(t(16, 16), t(3, 3))
    with pytest.raises(ValueError, match="device tensors"):
        rise.gemm_backward(t(8, 8), t(8, 8), t(8, 8))


def test_bf16_autograd_backward_widens_before_the_library():
    # RiseGemmFn saves bfloat16 operands in mode "bf16"; its backward widens them
    # to FP32 (exact) before gemm_backward, which only takes FP32.  On the host the
    # call stops at the device check, after the type check has passed.
    A = t(8, 8, dtype=torch.bfloat16)
    with pytest.raises(ValueError, match="device tensors"):
        rise.gemm_backward(t(8, 8), A.float(), t(8, 8))
