"""pcol_deposit_noalloc (the deposition on the library's fixed device scratch, with
no allocation) through the C ABI, against pcol_deposit (the context path) on the
same input: bitwise equal (same kernels and summation order; no element holds more
than 64 spheres here), and within the summation bound of the oracle's deposition.
Two calls in a row, the second with a smaller input, so anything the first left in
the shared scratch would show; an input too large for the scratch and a bad position
are refused with the output unchanged."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _case(n, seed, nc, comp):
    L = (3.0, 2.0, 5.0)
    x, y, z, a = workloads.deposit_case(n, seed=seed, L=L, comp=comp)
    return [_dev(v) for v in (x, y, z)] + [_dev(a)], (x, y, z, a), L


def _max_occupancy(host, nc, L):
    cells = [np.minimum(np.floor(p / (L[d] / nc[d])).astype(np.int64), nc[d] - 1)
             for d, p in enumerate(host[:3])]
    e = (cells[2] * nc[1] + cells[1]) * nc[0] + cells[0]
    return int(np.bincount(e, minlength=nc[0] * nc[1] * nc[2]).max()) if len(e) else 0


def _bitwise(got, ref, what):
    diff = int((got.view(torch.int64) != ref.view(torch.int64)).sum().item())
    assert diff == 0, f"{what}: {diff} values differ"


def _noalloc(args, nc, L, comp):
    x, y, z, a = args
    out = torch.full((nc[2], nc[1], nc[0], comp), 7.0, dtype=torch.float64, device="cuda")
    pc.pcol_deposit_noalloc(x, y, z, a, nc, L, out)
    torch.cuda.synchronize()
    return out


def _within_oracle(host, nc, L, got):
    x, y, z, a = host
    ref = oracle.deposit(x, y, z, a, nc, L)
    mag = oracle.deposit(x, y, z, np.abs(a), nc, L)
    g = np.ascontiguousarray(got.cpu().numpy().transpose(3, 0, 1, 2))
    # every node has at most 8 * (spheres of its elements) terms; bound by n
    k = len(x)
    assert np.all(np.abs(g - ref) <= 2.0 * (k - 1) * U * mag * (1 + 1e-6) + 0.0)


def test_noalloc_matches_pcol_deposit_on_two_calls_in_a_row():
    print("[gpu-test] pcol_deposit_noalloc: two calls, the second smaller", flush=True)
    ctx = pc.Context(1)
    for n, seed, nc, comp in ((200_000, 21, (40, 30, 50), 4), (50_000, 22, (17, 23, 11), 3)):
        args, host, L = _case(n, seed, nc, comp)
        assert _max_occupancy(host, nc, L) <= 64  # caller-index order in every element
        got = _noalloc(args, nc, L, comp)
        ref = pc.pcol_deposit(ctx, *args, nc, L)
        torch.cuda.synchronize()
        _bitwise(got, ref, f"n={n} nc={nc} comp={comp}")
        _within_oracle(host, nc, L, got)
    ctx.close()


def test_noalloc_on_a_side_stream_and_empty_input():
    print("[gpu-test] pcol_deposit_noalloc: side stream, n = 0", flush=True)
    nc, comp = (9, 8, 7), 2
    args, host, L = _case(3_000, 23, nc, comp)
    assert _max_occupancy(host, nc, L) <= 64
    ctx = pc.Context(1)
    ref = pc.pcol_deposit(ctx, *args, nc, L)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        out = torch.empty((nc[2], nc[1], nc[0], comp), dtype=torch.float64, device="cuda")
        pc.pcol_deposit_noalloc(*args, nc, L, out)
    side.synchronize()
    _bitwise(out, ref, "side stream")
    empty = [torch.empty(0, dtype=torch.float64, device="cuda") for _ in range(3)]
    a0 = torch.empty((comp, 0), dtype=torch.float64, device="cuda")
    z = _noalloc(empty + [a0], nc, L, comp)
    assert torch.count_nonzero(z).item() == 0
    ctx.close()


def test_noalloc_refuses_what_does_not_fit_and_bad_positions():
    print("[gpu-test] pcol_deposit_noalloc: refused inputs", flush=True)
    nc, comp = (256, 256, 160), 4  # 8 B per element alone: 84 MB > 64 MiB
    args, host, L = _case(1000, 24, nc, comp)
    out = torch.full((nc[2], nc[1], nc[0], comp), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_deposit_noalloc(*args, nc, L, out)
    assert ei.value.code == pc.PCOL_E_SCRATCH
    assert torch.all(out == 7.0).item()
    nc = (10, 10, 10)
    args, host, L = _case(5000, 25, nc, comp)
    args[1][17] = L[1]  # y == L: outside [0, L)
    out = torch.full((nc[2], nc[1], nc[0], comp), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(pc.PcolError) as ei:
        pc.pcol_deposit_noalloc(*args, nc, L, out)
    assert ei.value.code == pc.PCOL_E_INVALID
    torch.cuda.synchronize()
    assert torch.all(out == 7.0).item()
    # the scratch still serves a good call afterwards
    args[1][17] = 0.5
    assert _max_occupancy(host, nc, L) <= 64
    got = _noalloc(args, nc, L, comp)
    ctx = pc.Context(1)
    ref = pc.pcol_deposit(ctx, *args, nc, L)
    torch.cuda.synchronize()
    _bitwise(got, ref, "after a refused call")
    ctx.close()
