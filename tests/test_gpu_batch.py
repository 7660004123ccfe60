"""GPU parity of batched uneven solves (many independent densities, grid sides
128..2048, one launch per stage over all members) against the FP64 oracle and
against single-plan solves of the same members.

Bars: each member within the single-solve bars against the oracle (rel L-inf
and L2 <= 1e-10 FP64, <= 1e-6 FP32); every member bitwise equal to the same
density solved by a single plan (the batched kernels run the single-solve
kernel bodies at each member's length, so the arithmetic is the same)."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BARS = {torch.float64: 1e-10, torch.float32: 1e-6}
TOLS = {torch.float64: 1e-12, torch.float32: 1e-7}


def rel_linf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ps():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_2014_amd as ps
    return ps


def member_list(count, seed=1, sizes=None):
    """(n, half, density) of `count` batch members; `sizes` overrides the drawn sides."""
    out = []
    for i, (n, half, spec) in enumerate(W.batch_members(seed=seed, count=count)):
        if sizes is not None:
            n = sizes[i % len(sizes)]
            half = n / 64.0
        out.append((n, half, W.mixture_density(n, half, spec)))
    return out


def batch_params(members, dtype, **extra):
    return [dict(n=n, h=2 * half / n, n_r=64, n_theta=128, tol=TOLS[dtype], **extra) for n, half, _ in members]


def single_solves(ps, members, dtype, adjoint=False, inputs=None, sort=None):
    """Each member through a single plan of its own parameters (one plan per
    size); sort[i] = (bin, sub_nodes) of member i when not the defaults."""
    plans, outs = {}, []
    for i, (n, half, rho) in enumerate(members):
        extra = {} if sort is None else dict(bin=sort[i][0], sub_nodes=sort[i][1])
        key = (n, half, tuple(sorted(extra.items())))
        if key not in plans:
            plans[key] = ps.Plan(n, 2 * half / n, dtype=dtype, n_r=64, n_theta=128, tol=TOLS[dtype], **extra)
        src = torch.as_tensor(rho if inputs is None else inputs[i], dtype=dtype, device="cuda")
        fn = plans[key].solve_adjoint if adjoint else plans[key].solve
        outs.append(fn(src.contiguous()))
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in outs]
    for p in plans.values():
        p.close()
    return res


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_members_match_oracle_and_single_plans(ps, dtype):
    # two members of each supported side, in an order that is not by size
    sizes = [256, 128, 1024, 512, 2048, 128, 512, 256, 1024]
    members = member_list(len(sizes), seed=5, sizes=sizes)
    print(f"case: batch of {len(members)} sizes {sizes} {dtype}", flush=True)
    bp = ps.BatchPlan(batch_params(members, dtype), dtype=dtype)
    packed = bp.pack([m[2] for m in members])
    out = bp.solve(packed)
    torch.cuda.synchronize()
    got = [g.cpu().numpy() for g in bp.unpack(out)]
    used = [g.double().cpu().numpy() for g in bp.unpack(packed)]
    single = single_solves(ps, members, dtype, inputs=used)
    for i, (n, half, _) in enumerate(members):
        assert np.array_equal(got[i], single[i]), f"member {i} (N={n}) differs from its single-plan solve"
        if n <= 1024:
            ref = O.phi(used[i], O.SplitParams(n=n, h=2 * half / n, n_r=64, n_theta=128))
            assert rel_linf(got[i], ref) <= BARS[dtype], f"member {i} N={n}"
            assert rel_l2(got[i], ref) <= BARS[dtype], f"member {i} N={n}"
    bp.close()


@pytest.mark.parametrize("n,dtype", [(128, torch.float64), (2048, torch.float32)])
def test_one_member_batch_equals_single_plan(ps, n, dtype):
    """The degenerate batch of one member (the smallest and the largest side a
    batch takes): forward and transposed solves equal the single plan's bits."""
    members = member_list(1, seed=21, sizes=[n])
    print(f"case: one-member batch N={n} {dtype}", flush=True)
    bp = ps.BatchPlan(batch_params(members, dtype), dtype=dtype)
    packed = bp.pack([members[0][2]])
    used = [t.double().cpu().numpy() for t in bp.unpack(packed)]
    fwd = bp.unpack(bp.solve(packed))[0].cpu().numpy()
    back = bp.unpack(bp.solve_adjoint(packed))[0].cpu().numpy()
    assert np.array_equal(fwd, single_solves(ps, members, dtype, inputs=used)[0])
    assert np.array_equal(back, single_solves(ps, members, dtype, adjoint=True, inputs=used)[0])
    bp.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_adjoint_matches_single_plans_and_oracle(ps, dtype):
    sizes = [128, 512, 256, 128]
    members = member_list(len(sizes), seed=9, sizes=sizes)
    print(f"case: batch adjoint sizes {sizes} {dtype}", flush=True)
    rng = np.random.default_rng(17)
    g = [rng.standard_normal((n, n)) for n, _, _ in members]
    bp = ps.BatchPlan(batch_params(members, dtype), dtype=dtype)
    packed = bp.pack(g)
    back = bp.solve_adjoint(packed)
    torch.cuda.synchronize()
    got = [t.cpu().numpy() for t in bp.unpack(back)]
    used = [t.double().cpu().numpy() for t in bp.unpack(packed)]
    single = single_solves(ps, members, dtype, adjoint=True, inputs=used)
    for i, (n, half, _) in enumerate(members):
        assert np.array_equal(got[i], single[i]), f"member {i} (N={n})"
        ref = O.phi_transpose(used[i], O.SplitParams(n=n, h=2 * half / n, n_r=64, n_theta=128))
        e_inf, e_2 = rel_linf(got[i], ref), rel_l2(got[i], ref)
        print(f"  member {i} N={n}: rel L-inf {e_inf:.3e}, L2 {e_2:.3e}", flush=True)
        assert e_2 <= BARS[dtype], f"member {i} N={n}"
        assert e_inf <= BARS[dtype], f"member {i} N={n}"
    bp.close()


def test_full_uneven_batch_fp32(ps):
    """The 256-member batch with sides drawn from {128, 256, 512, 1024} at
    h = 1/32 and autotuned node sorts: every member bitwise equal to its
    single-plan solve with the same node sort, four members of each side
    against the oracle."""
    members = member_list(256, seed=1)
    print("case: 256-member uneven batch FP32, autotuned", flush=True)
    dtype = torch.float32
    bp = ps.BatchPlan(batch_params(members, dtype, autotune=True), dtype=dtype)
    sort = []
    for i in range(len(members)):
        info = bp.member_info(i)
        assert info["n"] == members[i][0]
        sort.append((info["bin"], info["sub_nodes"]))
    print("chosen node sorts by side:", sorted(set((m[0],) + s for m, s in zip(members, sort))), flush=True)
    packed = bp.pack([m[2] for m in members])
    out = bp.solve(packed)
    torch.cuda.synchronize()
    got = [g.cpu().numpy() for g in bp.unpack(out)]
    used = [g.double().cpu().numpy() for g in bp.unpack(packed)]
    single = single_solves(ps, members, dtype, inputs=used, sort=sort)
    bad = [i for i in range(len(members)) if not np.array_equal(got[i], single[i])]
    assert not bad, f"members {bad[:8]} differ from their single-plan solves"
    checked = {}
    for i, (n, half, _) in enumerate(members):
        if checked.get(n, 0) >= 4:
            continue
        checked[n] = checked.get(n, 0) + 1
        ref = O.phi(used[i], O.SplitParams(n=n, h=2 * half / n, n_r=64, n_theta=128))
        assert rel_linf(got[i], ref) <= 1e-6, f"member {i} N={n}"
        assert rel_l2(got[i], ref) <= 1e-6, f"member {i} N={n}"
    assert checked == {128: 4, 256: 4, 512: 4, 1024: 4}
    bp.close()


def test_members_differing_only_in_node_sort_keep_their_own(ps):
    """Two members with equal parameters except the requested node sort: each
    keeps its own bin side and subproblem size, and each equals the single plan
    of its own parameters bit for bit."""
    sizes = [256, 256, 256]
    members = member_list(len(sizes), seed=4, sizes=sizes)
    sort = [(4, 64), (8, 32), (4, 64)]
    print("case: batch members differing in node sort", flush=True)
    dtype = torch.float32
    params = [dict(p, bin=b, sub_nodes=sn) for p, (b, sn) in zip(batch_params(members, dtype), sort)]
    bp = ps.BatchPlan(params, dtype=dtype)
    for i, (b, sn) in enumerate(sort):
        info = bp.member_info(i)
        assert (info["bin"], info["sub_nodes"]) == (b, sn), f"member {i}"
    packed = bp.pack([m[2] for m in members])
    got = [g.cpu().numpy() for g in bp.unpack(bp.solve(packed))]
    used = [g.double().cpu().numpy() for g in bp.unpack(packed)]
    single = single_solves(ps, members, dtype, inputs=used, sort=sort)
    for i in range(len(members)):
        assert np.array_equal(got[i], single[i]), f"member {i}"
    bp.close()


def test_batch_graph_replay_matches_eager(ps):
    sizes = [512, 128, 256]
    members = member_list(len(sizes), seed=3, sizes=sizes)
    print("case: batch graph replay", flush=True)
    dtype = torch.float32
    bp = ps.BatchPlan(batch_params(members, dtype), dtype=dtype)
    packed = bp.pack([m[2] for m in members])
    eager = bp.solve(packed).clone()
    out = torch.empty_like(packed)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bp.solve(packed, out)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bp.solve(packed, out)
    ref = eager.cpu().numpy()
    for _ in range(3):
        out.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref)
        bp.solve(packed, eager)
        torch.cuda.synchronize()
    bp.close()


def test_batch_argument_errors(ps):
    from paper_1409_2014_amd import _binding as B
    print("case: batch argument errors", flush=True)
    good = dict(n=128, h=1 / 32)
    with pytest.raises(B.PhiError, match="PHI_ERR_UNSUPPORTED"):
        ps.BatchPlan([good, dict(n=64, h=1 / 32)], dtype=torch.float32)
    # mixed data precision is refused
    p32 = ps.make_params(128, 1 / 32, dtype=torch.float32)
    p64 = ps.make_params(128, 1 / 32, dtype=torch.float64)
    arr = (B.PhiParams * 2)(p32, p64)
    h = ctypes.c_void_p()
    st = B.lib().phi_plan_batch(arr, 2, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    assert B.STATUS_NAMES[st] == "PHI_ERR_INVALID_ARG"
    # stage entry points take single plans only
    bp = ps.BatchPlan([good, good], dtype=torch.float32)
    src = torch.zeros(bp.total, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    st = B.lib().phi_solve_highfreq(bp._handle, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert B.STATUS_NAMES[st] == "PHI_ERR_UNSUPPORTED"
    assert bp.offsets == [0, 128 * 128, 2 * 128 * 128]
    bp.close()
