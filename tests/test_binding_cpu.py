"""CPU tests of the Python binding's argument marshalling (no GPU calls)."""
import torch

from paper_2604_16590_amd import _binding as b


def test_dense_layout_detection():
    x = torch.empty(2, 3, 5, 8)
    assert b._dense(x)
    assert b._dense(x.permute(0, 2, 1, 3))            # BNHD view: dense, reordered
    assert b._dense(torch.empty(1, 1, 7, 4))
    assert not b._dense(x[:, :, ::2])                  # gaps
    assert not b._dense(torch.ones(1).expand(2, 3, 5, 8))  # o.sum()'s gradient: strides 0
    assert not b._dense(torch.empty(2, 1, 5, 8).expand(2, 3, 5, 8))


def test_autograd_gradient_layouts_reach_q_layout(monkeypatch):
    # The autograd backward must hand la_backward a dO with q's dtype and
    # strides whatever layout autograd passes; the C call is replaced by a
    # recorder so this runs without a GPU.
    seen = {}

    def fake_backward(q, k, v, S, z, dout, grad_dtype=None):
        seen["q"], seen["do"] = q, dout
        return torch.zeros_like(q), torch.zeros_like(k), torch.zeros_like(v)

    monkeypatch.setattr(b, "backward", fake_backward)

    class Ctx:
        def __init__(self, *t):
            self.saved_tensors = t

    q = torch.randn(2, 3, 5, 8).to(torch.bfloat16)
    S, z = torch.zeros(2, 3, 8, 8, dtype=torch.float64), torch.zeros(2, 3, 8, dtype=torch.float64)
    cases = [
        torch.ones((), dtype=torch.bfloat16).expand(2, 3, 5, 8),       # o.sum()
        torch.randn(2, 5, 3, 8).to(torch.bfloat16).permute(0, 2, 1, 3),  # transposed storage
        torch.randn(2, 3, 8, 5).to(torch.bfloat16).transpose(2, 3),      # feature stride != 1
        torch.randn(2, 3, 5, 8),                                          # fp32 gradient
    ]
    for g in cases:
        b.LinearAttention.backward(Ctx(q, q, q, S, z), g)
        do = seen["do"]
        assert do.dtype == q.dtype and do.stride() == seen["q"].stride()
        assert torch.equal(do.float(), g.to(q.dtype).float())
    # a broadcast q (strides 0): everything goes dense
    qb = torch.randn(1, 3, 5, 8).to(torch.bfloat16).expand(2, 3, 5, 8)
    b.LinearAttention.backward(Ctx(qb, qb, qb, S, z), cases[1])
    assert seen["q"].is_contiguous() and seen["do"].is_contiguous()
