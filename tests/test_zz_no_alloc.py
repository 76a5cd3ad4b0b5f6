"""The no-allocation entry point rbws_exact_dots_noalloc, through the C ABI.

It must give the same correctly rounded dots as rbws_exact_dots, bit for bit,
on two calls in a row (the second with a smaller input, so that the shared
workspace holds the first call's partial sums when the second starts), write
zeros for empty vectors, and reject inputs whose partial sums exceed its fixed
workspace with EINVAL before anything is launched.
"""
import ctypes as C

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    from paper_2311_13862_amd import rbws
    assert torch.cuda.is_available()
    return rbws


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def pair(rng, count, length, scale_exp):
    s = 10.0 ** rng.uniform(-scale_exp, scale_exp, (count, length))
    x = rng.standard_normal((count, length)) * s
    y = rng.standard_normal((count, length)) / s
    y[:, 1::3] = -x[:, 1::3]  # heavy cancellation
    return x, y


@pytest.mark.parametrize("flags", [0, 1])
def test_noalloc_dots_equal_allocating_entry_point(rb, flags):
    rng = np.random.default_rng(11 + flags)
    # first call: 6 vectors of a ragged length that spans 74 partial sums each;
    # second call: fewer, shorter vectors (3 x 12345, 4 partial sums each)
    for count, length, sexp in ((6, 300_001, 40), (3, 12_345, 3)):
        x, y = pair(rng, count, length, sexp)
        X, Y = dev(x), dev(y)
        want = rb.exact_dots(X, Y, flags=flags)
        out = torch.full((count,), float("nan"), dtype=torch.float64, device="cuda")
        rb.exact_dots_noalloc(X, Y, out, flags=flags)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, want), (count, length, got, want)
        for b in range(count):
            assert got[b] == oracle.exact_dot(x[b], y[b]), (count, length, b)


def test_noalloc_dots_on_a_side_stream(rb):
    """Stream-ordered: the result is there once the caller's stream is done."""
    rng = np.random.default_rng(5)
    x, y = pair(rng, 4, 65_536 + 3, 5)
    X, Y = dev(x), dev(y)
    want = rb.exact_dots(X, Y)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        rb.exact_dots_noalloc(X, Y, out, stream=st)
    st.synchronize()
    assert np.array_equal(out.cpu().numpy(), want)


def test_noalloc_dots_empty_and_limits(rb):
    L = rb.lib()
    out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    x = torch.zeros((3, 8), dtype=torch.float64, device="cuda")
    # length 0: exact zeros
    assert L.rbws_exact_dots_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), 0, 3,
                                     C.c_void_p(out.data_ptr()), 0, None) == rb.OK
    torch.cuda.synchronize()
    assert out.cpu().numpy().tolist() == [0.0, 0.0, 0.0]
    # count 0: nothing to do
    assert L.rbws_exact_dots_noalloc(None, None, 5, 0, None, 0, None) == rb.OK
    # more partial sums than the workspace holds: rejected on the host, nothing
    # is launched (the vectors are never read, so a short buffer is safe here)
    cap = rb.NOALLOC_SCRATCH_BYTES // rb.NOALLOC_PARTIAL_BYTES
    too_long = 4096 * (cap // 2 + 1)
    assert L.rbws_exact_dots_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), too_long, 2,
                                     C.c_void_p(out.data_ptr()), 0, None) == rb.EINVAL
    assert b"workspace" in L.rbws_last_error()
    # NULL output
    assert L.rbws_exact_dots_noalloc(C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), 8, 3, None, 0,
                                     None) == rb.EINVAL
