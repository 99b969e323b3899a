"""pcol_deposit on the GPU against the oracle's orc_deposit, node by node.

The weights are computed by the same binary64 formulas on both sides, so a node
that receives a single contribution is compared bitwise.  The other node sums are
associated differently (the GPU sums per element, then over a node's eight
elements; the oracle over all spheres in index order), and each must lie within
2 (k - 1) 2^-53 sum|w a| of the oracle's: both are within (k - 1) 2^-53 sum|w a|
of the exact sum, k the node's number of contributions.  Repeated calls agree
bitwise."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2501_05340_amd as pc  # noqa: E402  (no CPU fallback: a missing library fails)

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _announce(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def gpu_deposit(x, y, z, a, nc, L, ctx=None):
    ctx = ctx or pc.Context(1)
    out = pc.pcol_deposit(ctx, _dev(x), _dev(y), _dev(z), _dev(a), nc, L)
    torch.cuda.synchronize()
    # node-major (nc2, nc1, nc0, comp) -> the oracle's (comp, nc2, nc1, nc0)
    return np.ascontiguousarray(out.cpu().numpy().transpose(3, 0, 1, 2))


def contributions(x, y, z, nc, L):
    """Number of spheres depositing on each node, shape (nc2, nc1, nc0) (for the
    tolerance only)."""
    nodes = []
    for p, d in ((x, 0), (y, 1), (z, 2)):
        s = p / (L[d] / nc[d])
        c = np.minimum(np.floor(s).astype(np.int64), nc[d] - 1)
        nodes.append((c, (c + 1) % nc[d]))
    cnt = np.zeros(nc[0] * nc[1] * nc[2], dtype=np.int64)
    for b in range(8):
        i = nodes[0][b & 1]
        j = nodes[1][(b >> 1) & 1]
        k = nodes[2][(b >> 2) & 1]
        np.add.at(cnt, (k * nc[1] + j) * nc[0] + i, 1)
    return cnt.reshape(nc[2], nc[1], nc[0])


def check(x, y, z, a, nc, L, got):
    ref = oracle.deposit(x, y, z, a, nc, L)
    mag = oracle.deposit(x, y, z, np.abs(a), nc, L)
    k = contributions(x, y, z, nc, L)[None]
    tol = 2.0 * np.maximum(k - 1, 0) * U * mag * (1.0 + 1e-6)
    err = np.abs(got - ref)
    assert np.all(err <= tol), f"max excess {np.max(err - tol):.3e}"
    single = np.broadcast_to(k <= 1, ref.shape)
    assert np.array_equal(got[single].view(np.uint64), ref[single].view(np.uint64)), \
        "a node with one contribution differs bitwise"
    return int(np.count_nonzero(k > 1))


@pytest.mark.parametrize("n,nc,comp", [(1, (4, 5, 6), 4), (65, (7, 5, 3), 1), (4097, (16, 16, 16), 4),
                                        (20000, (31, 17, 9), 3), (19963, (40, 40, 40), 8),
                                        (100000, (1, 3, 64), 2)])
def test_deposit_matches_oracle(n, nc, comp):
    L = (1.3, 0.9, 2.1)
    _announce(f"deposit n={n} nc={nc} comp={comp}")
    x, y, z, a = workloads.deposit_case(n, seed=n, L=L, comp=comp)
    got = gpu_deposit(x, y, z, a, nc, L)
    check(x, y, z, a, nc, L, got)


def test_deposit_sparse_is_bitwise():
    # at most one sphere per cell corner neighbourhood: every node sum has one term
    nc, L = (64, 64, 64), (1.0, 1.0, 1.0)
    g = np.arange(0, 64, 2) / 64.0 + 1.0 / 128.0
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = xx.ravel(), yy.ravel(), zz.ravel()
    rng = np.random.default_rng(4)
    x = x + rng.uniform(-1, 1, x.size) / 300.0
    a = rng.normal(size=(4, x.size))
    _announce(f"deposit sparse n={x.size}")
    got = gpu_deposit(x, y, z, a, nc, L)
    ref = oracle.deposit(x, y, z, a, nc, L)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_deposit_edges_and_wrap():
    # spheres on nodes, at 0, just below L, and in the last cell of every axis
    nc, L = (4, 4, 4), (1.0, 2.0, 0.5)
    below = [np.nextafter(v, 0.0) for v in L]
    x = np.array([0.0, below[0], 0.25, 0.875, below[0]])
    y = np.array([0.0, below[1], 1.0, 1.75, 0.0])
    z = np.array([0.0, below[2], 0.125, 0.4375, below[2]])
    a = np.arange(10, dtype=np.float64).reshape(2, 5) + 1.0
    _announce("deposit edges")
    got = gpu_deposit(x, y, z, a, nc, L)
    check(x, y, z, a, nc, L, got)


def test_deposit_empty_and_conservation():
    _announce("deposit empty")
    ctx = pc.Context(1)
    nc, L = (3, 3, 3), (1.0, 1.0, 1.0)
    out = torch.full((3, 3, 3, 4), float("nan"), dtype=torch.float64, device="cuda")
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    pc.pcol_deposit(ctx, e, e, e, torch.empty((4, 0), dtype=torch.float64, device="cuda"), nc, L,
                    out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    x, y, z, a = workloads.deposit_case(50000, seed=9, L=L, comp=4)
    got = gpu_deposit(x, y, z, a, (10, 10, 10), L, ctx)
    s = got.reshape(4, -1).sum(axis=1)
    np.testing.assert_allclose(s, a.sum(axis=1), rtol=0, atol=1e-9)


def test_deposit_errors_leave_output_unchanged():
    _announce("deposit errors")
    ctx = pc.Context(1)
    nc, L = (4, 4, 4), (1.0, 1.0, 1.0)
    x, y, z, a = workloads.deposit_case(1000, seed=3, L=L, comp=4)
    out = torch.full((4, 4, 4, 4), 7.0, dtype=torch.float64, device="cuda")
    for bad in (1.0, -1e-300, float("nan"), float("inf")):
        xb = x.copy()
        xb[517] = bad
        with pytest.raises(pc.PcolError) as ei:
            pc.pcol_deposit(ctx, _dev(xb), _dev(y), _dev(z), _dev(a), nc, L, out)
        assert ei.value.code == pc.PCOL_E_INVALID
        torch.cuda.synchronize()
        assert torch.all(out == 7.0).item()
    for kw in ({"nc": (0, 4, 4)}, {"L": (1.0, -1.0, 1.0)}):
        args = {"nc": nc, "L": L, **kw}
        with pytest.raises(pc.PcolError):
            pc.pcol_deposit(ctx, _dev(x), _dev(y), _dev(z), _dev(a), args["nc"], args["L"],
                            torch.empty(int(np.prod(args["nc"])) * 4, dtype=torch.float64,
                                        device="cuda"))
    a9 = np.zeros((9, 1000))
    with pytest.raises(pc.PcolError):
        pc.pcol_deposit(ctx, _dev(x), _dev(y), _dev(z), _dev(a9), nc, L)
    assert torch.all(out == 7.0).item()


def test_deposit_repeats_bitwise_and_dense_elements():
    L = (1.0, 1.0, 1.0)
    x, y, z, a = workloads.deposit_case(200_000, seed=21, L=L, comp=4)
    ctx = pc.Context(1)
    _announce("deposit repeat")
    one = gpu_deposit(x, y, z, a, (24, 24, 24), L, ctx)
    two = gpu_deposit(x, y, z, a, (24, 24, 24), L, ctx)
    assert np.array_equal(one.view(np.uint64), two.view(np.uint64))
    check(x, y, z, a, (24, 24, 24), L, one)
    # 2 x 3 x 2 elements of about 17,000 spheres each: sums in scatter order
    _announce("deposit dense elements")
    check(x, y, z, a, (2, 3, 2), L, gpu_deposit(x, y, z, a, (2, 3, 2), L, ctx))
    # a smaller call after the larger ones reuses the grown scratch
    check(x[:999], y[:999], z[:999], a[:, :999].copy(), (5, 4, 3), L,
          gpu_deposit(x[:999], y[:999], z[:999], a[:, :999].copy(), (5, 4, 3), L, ctx))


def _ordered_reference(x, y, z, a, nc, L):
    """The node sums in the association the header states: per element, w a summed
    over its spheres in caller-index order; per node, the eight corner sums in the
    order b = 0..7 (plain Python floats: binary64, no contraction)."""
    comp, n = a.shape
    h = [L[d] / nc[d] for d in range(3)]
    E = {}
    for i in range(n):
        c, f = [], []
        for d, p in enumerate((x[i], y[i], z[i])):
            s = float(p) / h[d]
            cd = min(int(np.floor(s)), nc[d] - 1)
            c.append(cd)
            f.append(s - cd)
        e = (c[2] * nc[1] + c[1]) * nc[0] + c[0]
        acc = E.setdefault(e, [[0.0] * comp for _ in range(8)])
        for b in range(8):
            w = (((f[0] if b & 1 else 1.0 - f[0]) * (f[1] if b & 2 else 1.0 - f[1]))
                 * (f[2] if b & 4 else 1.0 - f[2]))
            for q in range(comp):
                acc[b][q] += w * float(a[q, i])
    out = np.zeros((comp, nc[2], nc[1], nc[0]))
    zero = [[0.0] * comp for _ in range(8)]
    for k in range(nc[2]):
        for j in range(nc[1]):
            for i in range(nc[0]):
                sq = [0.0] * comp
                for b in range(8):
                    ei = (i - (b & 1)) % nc[0]
                    ej = (j - ((b >> 1) & 1)) % nc[1]
                    ek = (k - ((b >> 2) & 1)) % nc[2]
                    src = E.get((ek * nc[1] + ej) * nc[0] + ei, zero)
                    for q in range(comp):
                        sq[q] += src[b][q]
                out[:, k, j, i] = sq
    return out


@pytest.mark.parametrize("n,nc", [(30000, (16, 16, 16)), (30000, (12, 10, 9))])
def test_deposit_summation_order_bitwise(n, nc):
    # 7 to 28 spheres per element: both the register and the memory selection
    L = (1.0, 0.8, 1.3)
    x, y, z, a = workloads.deposit_case(n, seed=n + nc[1], L=L, comp=2)
    _announce(f"deposit order n={n} nc={nc}")
    got = gpu_deposit(x, y, z, a, nc, L)
    ref = _ordered_reference(x, y, z, a, nc, L)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    check(x, y, z, a, nc, L, got)


def test_deposit_full_size_16M():
    """The bench workload's shape: 16M spheres uniform in the box on 160^3 elements
    (3.9 spheres per element), four source components, every node against the oracle."""
    n, nc, L = 16_000_000, (160, 160, 160), (1.0, 1.0, 1.0)
    x, y, z, a = workloads.deposit_case(n, seed=3, L=L, comp=4)
    _announce(f"deposit full n={n} nc={nc}")
    got = gpu_deposit(x, y, z, a, nc, L)
    multi = check(x, y, z, a, nc, L, got)
    assert multi > 1_000_000
