"""torch.autograd.Function wrappers: forward and backward both run the library's
HIP kernels (rise_gemm / rise_gemm_backward, rise_stencil2d /
rise_stencil2d_backward); torch only supplies device memory and the stream."""
import torch


class RiseGemmFn(torch.autograd.Function):
    """C = A . B (FP32 row-major), gradients dA = dC B^T, dB = A^T dC."""

    @staticmethod
    def forward(ctx, A, B, mode="f32"):
        from . import gemm

        ctx.save_for_backward(A, B)
        ctx.mode = mode
        return gemm(A, B, mode=mode)

    @staticmethod
    def backward(ctx, dC):
        from . import gemm_backward

        A, B = ctx.saved_tensors
        # the backward products read FP32 operands; bfloat16 operands (mode "bf16")
        # widen exactly, and each gradient is returned in its operand's type
        dA, dB = gemm_backward(dC.float(), A.float(), B.float(), mode=ctx.mode,
                               need_dA=ctx.needs_input_grad[0],
                               need_dB=ctx.needs_input_grad[1])
        if dA is not None:
            dA = dA.to(A.dtype)
        if dB is not None:
            dB = dB.to(B.dtype)
        return dA, dB, None


class RiseStencil2dFn(torch.autograd.Function):
    """out = stencil(img, w) with clamp or zero padding; gradients for img and w."""

    @staticmethod
    def forward(ctx, img, w, pad="clamp"):
        from . import stencil2d

        ctx.save_for_backward(img, w)
        ctx.pad = pad
        return stencil2d(img, w, pad=pad)

    @staticmethod
    def backward(ctx, dOut):
        from . import stencil2d_backward

        img, w = ctx.saved_tensors
        dIn, dW = stencil2d_backward(dOut, img, w, pad=ctx.pad,
                                     need_din=ctx.needs_input_grad[0],
                                     need_dw=ctx.needs_input_grad[1])
        return dIn, dW, None


class RiseConv2dFn(torch.autograd.Function):
    """Stencil layer: bfloat16 NHWC activations, FP32 weights, 3 x 3, zero padding."""

    @staticmethod
    def forward(ctx, x, w):
        from . import conv2d

        ctx.save_for_backward(x, w)
        return conv2d(x, w, pad="zero")

    @staticmethod
    def backward(ctx, dOut):
        from . import conv2d_backward

        x, w = ctx.saved_tensors
        dIn, dW = conv2d_backward(dOut.to(torch.bfloat16), x, w, pad="zero",
                                  need_din=ctx.needs_input_grad[0],
                                  need_dw=ctx.needs_input_grad[1])
        return dIn, dW
