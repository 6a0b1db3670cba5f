"""The streaming probes behind the roofline ceilings (lb_probe_stream) move
what they claim: the copy kernel reproduces its source bit for bit, the
write kernel fills every 16-byte chunk with its pattern, the read kernel
leaves the destination alone for finite inputs, and the collide-pattern
kernel stores at node n of plane (k, i) the value of node n - c_i (D3Q19,
periodic, in the library's direction order from lb_lattice). The z-march
kernel stores that value plus 1e-3 sum_j j s_{1-k}(n + c_j), s the per-node
sums of the pulled values, on boxes of one and of several column tiles and
plane chunks. Sizes are chosen off the workgroup and chunk multiples so that
the tails are covered."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import requires_gpu

pytestmark = [pytest.mark.gpu, requires_gpu]


def _probe(kind, src, dst, nbytes, box=(0, 0, 0)):
    import torch
    from paper_2004_04080_amd import binding as B
    ms = C.c_double()
    B.check(B.lib().lb_probe_stream(kind, C.c_void_p(src.data_ptr() if src is not None else 0),
                                    C.c_void_p(dst.data_ptr()), nbytes, *box, 1,
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                    C.byref(ms)), "lb_probe_stream")
    torch.cuda.synchronize()
    assert ms.value > 0.0


def test_copy_write_read_probes():
    import torch
    rng = np.random.default_rng(7)
    n16 = 1000 * 64 + 37                      # 16-byte chunks, not a multiple of a workgroup
    a_h = rng.standard_normal(4 * n16).astype(np.float32)
    a = torch.tensor(a_h, device="cuda:0")
    b = torch.full_like(a, -7.0)
    _probe(2, a, b, 16 * n16)
    assert np.array_equal(b.cpu().numpy().view(np.uint32), a_h.view(np.uint32))
    # write: chunk t holds (t mod 8, 1, 2, 3)
    c = torch.full((4 * n16 + 4,), -7.0, dtype=torch.float32, device="cuda:0")
    _probe(1, None, c, 16 * n16)
    got = c.cpu().numpy()
    want = np.stack([np.arange(n16) % 8, np.ones(n16), 2 * np.ones(n16), 3 * np.ones(n16)], 1)
    assert np.array_equal(got[:4 * n16].reshape(n16, 4), want.astype(np.float32))
    assert np.all(got[4 * n16:] == -7.0)          # nothing past the last chunk
    # read: finite inputs never reach the sink, so the destination stays as it was
    d = torch.full_like(a, -7.0)
    _probe(0, a, d, 16 * n16)
    assert np.all(d.cpu().numpy() == -7.0)


@pytest.mark.parametrize("box", [(13, 7, 5), (64, 3, 4)])
def test_collide_pattern_probe_is_the_pull_gather(box):
    import torch
    from paper_2004_04080_amd import binding as B
    nx, ny, nz = box
    N = nx * ny * nz
    c = (C.c_int32 * 57)()
    w = (C.c_double * 19)()
    B.check(B.lib().lb_lattice(c, w), "lb_lattice")
    cv = np.array(list(c), dtype=np.int64).reshape(19, 3)
    rng = np.random.default_rng(11)
    src_h = rng.standard_normal((2, 19, N)).astype(np.float32)
    src = torch.tensor(src_h.ravel(), device="cuda:0")
    dst = torch.full_like(src, np.nan)
    _probe(3, src, dst, src.numel() * 4, box)
    got = dst.cpu().numpy().reshape(2, 19, N)
    n = np.arange(N)
    x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)
    for i in range(19):
        m = ((x - cv[i, 0]) % nx) + nx * (((y - cv[i, 1]) % ny) + ny * ((z - cv[i, 2]) % nz))
        for k in range(2):
            assert np.array_equal(got[k, i], src_h[k, i, m]), (k, i)


def _lattice_c():
    from paper_2004_04080_amd import binding as B
    c = (C.c_int32 * 57)()
    w = (C.c_double * 19)()
    B.check(B.lib().lb_lattice(c, w), "lb_lattice")
    return np.array(list(c), dtype=np.int64).reshape(19, 3)


@pytest.mark.parametrize("box", [(128, 8, 3), (256, 16, 130)])
def test_march_pattern_probe(box):
    import torch
    nx, ny, nz = box
    N = nx * ny * nz
    cv = _lattice_c()
    rng = np.random.default_rng(13)
    src_h = rng.standard_normal((2, 19, N)).astype(np.float32)
    src = torch.tensor(src_h.ravel(), device="cuda:0")
    dst = torch.full_like(src, np.nan)
    _probe(4, src, dst, src.numel() * 4, box)
    got = dst.cpu().numpy().reshape(2, 19, N)
    n = np.arange(N)
    x, y, z = n % nx, (n // nx) % ny, n // (nx * ny)

    def shift(c):
        return ((x + c[0]) % nx) + nx * (((y + c[1]) % ny) + ny * ((z + c[2]) % nz))

    g = np.stack([np.stack([src_h[k, i, shift(-cv[i])] for i in range(19)]) for k in range(2)])
    g64 = g.astype(np.float64)
    s = g64.sum(axis=1)                          # [2, N], the per-node sums
    want = np.empty_like(g64)
    for k in range(2):
        st = sum(j * s[1 - k][shift(cv[j])] for j in range(1, 19))
        want[k] = g64[k] + 1e-3 * st[None, :]
    err = np.abs(got - want).max()
    print(f"[probe] march {box}: max |dst - reference| {err:.1e}", flush=True)
    assert np.isfinite(got).all() and err < 2e-5


def test_march_pattern_probe_rejects_other_shapes():
    import torch
    from paper_2004_04080_amd import binding as B
    a = torch.zeros(2 * 19 * 120 * 8 * 3, dtype=torch.float32, device="cuda:0")
    ms = C.c_double()
    rc = B.lib().lb_probe_stream(4, C.c_void_p(a.data_ptr()), C.c_void_p(a.data_ptr()),
                                 a.numel() * 4, 120, 8, 3, 1,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(ms))
    assert rc == B.LB_E_SHAPE
