"""Host logic of the Python binding (no GPU): the strides handed to the C ABI
for broadcast or single-row inputs, and the gradient plumbing of the autograd
wrappers for scalars given as numbers or tensors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2311_17189_amd import _lib  # noqa: E402
from paper_2311_17189_amd import autograd as ag  # noqa: E402


def test_broadcast_energies_are_copied():
    row = torch.arange(5, dtype=torch.float64).reshape(1, 5)
    e = row.expand(7, 5)                      # stride (0, 1): one row in memory
    t, st_s, st_i = _lib._energy_strides(e)
    assert (st_s, st_i) == (5, 1) and t.is_contiguous() and torch.equal(t, e)
    col = torch.arange(7, dtype=torch.float64).reshape(7, 1).expand(7, 5)   # stride (1, 0)
    t, st_s, st_i = _lib._energy_strides(col)
    assert (st_s, st_i) == (5, 1) and torch.equal(t, col)


def test_strides_passed_through_or_irrelevant():
    base = torch.zeros((9, 12), dtype=torch.float64)
    v = base[::2, 1:6]                        # strides (24, 1): passed as they are
    t, st_s, st_i = _lib._energy_strides(v)
    assert t.data_ptr() == v.data_ptr() and (st_s, st_i) == (24, 1)
    tr = base.t()[:5]                         # transposed view (1, 12)
    t, st_s, st_i = _lib._energy_strides(tr)
    assert t.data_ptr() == tr.data_ptr() and (st_s, st_i) == (1, 12)
    one = torch.zeros((1, 5), dtype=torch.float64).expand(1, 5)
    t, st_s, st_i = _lib._energy_strides(one)
    assert t.data_ptr() == one.data_ptr() and st_s >= 1 and st_i == 1
    single_col = torch.zeros((4, 1), dtype=torch.float64)
    assert _lib._energy_strides(single_col)[1:] == (1, 1)


def test_broadcast_momenta_are_copied():
    k0 = torch.arange(6, dtype=torch.float64).reshape(1, 6)
    k = k0.expand(4, 6)
    t, st = _lib._momentum_rows(k, 3)
    assert st == 6 and t.is_contiguous() and torch.equal(t, k)
    wide = torch.zeros((4, 10), dtype=torch.float64)[:, :6]
    t, st = _lib._momentum_rows(wide, 3)
    assert t.data_ptr() == wide.data_ptr() and st == 10
    t, st = _lib._momentum_rows(k0, 3)
    assert t.data_ptr() == k0.data_ptr() and st == 6


class _FakeAdjoint:
    """Stands in for the library calls: records the scalars they receive and
    returns gradients of the right shapes on the CPU."""

    def __init__(self):
        self.calls = []

    def forward(self, terms, k, q, t, mu, w, beta, e_reg, want_out, want_sum):
        self.calls.append(("fwd", t, mu, beta))
        return (torch.zeros((w.shape[0], k.shape[0]), dtype=torch.complex128),
                torch.zeros((w.shape[0],), dtype=torch.complex128))

    def adjoint(self, terms, k, q, t, mu, w, beta, e_reg, grad_out, grad_sum):
        self.calls.append(("adj", t, mu, beta))
        s = torch.tensor([1.0, 2.0, 3.0], dtype=torch.float64)
        return (torch.ones_like(k), s[0], s[1], s[2], torch.zeros((w.shape[0], 1), dtype=torch.complex128))


def _patch(monkeypatch):
    f = _FakeAdjoint()
    monkeypatch.setattr(ag, "evaluate_hubbard", f.forward)
    monkeypatch.setattr(ag, "evaluate_hubbard_adjoint", f.adjoint)
    return f


def test_hubbard_number_scalars_get_no_gradient(monkeypatch):
    f = _patch(monkeypatch)
    k = torch.zeros((3, 4), dtype=torch.float64, requires_grad=True)
    w = torch.zeros((2, 1), dtype=torch.complex128)
    out, s = ag.AmiHubbard.apply(None, k, np.zeros(2), 1.0, 0.25, w, 5.0)
    (out.real.sum() + s.real.sum()).backward()
    assert torch.equal(k.grad, torch.ones_like(k))
    assert [c[1:] for c in f.calls] == [(1.0, 0.25, 5.0), (1.0, 0.25, 5.0)]


def test_hubbard_tensor_scalars_get_gradients_on_their_devices(monkeypatch):
    _patch(monkeypatch)
    k = torch.zeros((3, 4), dtype=torch.float64, requires_grad=True)
    w = torch.zeros((2, 1), dtype=torch.complex128, requires_grad=True)
    t = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(0.1, dtype=torch.float64)               # no gradient asked
    beta = torch.tensor(4.0, dtype=torch.float64, requires_grad=True)
    out, s = ag.AmiHubbard.apply(None, k, np.zeros(2), t, mu, w, beta)
    s.real.sum().backward()
    assert float(t.grad) == 2.0 and float(beta.grad) == 3.0 and mu.grad is None
    assert t.grad.shape == t.shape and w.grad.shape == w.shape


def test_complex_energy_function_passes_gradients_through(monkeypatch):
    """AmiEvaluateComplex hands torch the adjoint's complex energy gradient as
    it is (torch's convention for complex inputs), a number beta gets none."""
    calls = []

    def fwd(terms, E, w, beta, e_reg, want_out=True, want_sum=True):
        calls.append(("fwd", beta))
        return torch.zeros((w.shape[0], E.shape[0]), dtype=torch.complex128), torch.zeros(w.shape[0],
                                                                                          dtype=torch.complex128)

    def adj(terms, E, w, beta, e_reg, grad_out=None, grad_sum=None):
        calls.append(("adj", beta))
        return torch.full_like(E, 2.0 - 1.0j), torch.tensor(3.0, dtype=torch.float64), torch.zeros_like(w)

    monkeypatch.setattr(ag, "evaluate_complex", fwd)
    monkeypatch.setattr(ag, "evaluate_complex_adjoint", adj)
    E = torch.zeros((3, 2), dtype=torch.complex128, requires_grad=True)
    w = torch.zeros((2, 1), dtype=torch.complex128)
    out, s = ag.AmiEvaluateComplex.apply(None, E, w, 5.0)
    (out.real.sum() + s.real.sum()).backward()
    assert torch.equal(E.grad, torch.full_like(E, 2.0 - 1.0j))
    assert calls == [("fwd", 5.0), ("adj", 5.0)]
