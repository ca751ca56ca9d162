"""Mixed-class plans (one persistent launch) against the oracle, against
eri4_batch, and under HIP-graph capture."""
import numpy as np
import pytest

import oracle
from paper_2307_03452_amd import eri4, inputs

pytestmark = pytest.mark.gpu
TOL = 1e-12
ZERO_SCALE = 1e-250


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    eri4.init()
    return _t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mixed(nq, seed, lvals, kmax):
    b = inputs.uneven_batch(nq=nq, seed=seed, lvals=lvals, kmax=kmax)
    return b


def oracle_blocks(b, idx):
    """Oracle result for quartets idx (grouped by class)."""
    res = {}
    by_cls = {}
    for q in idx:
        by_cls.setdefault(tuple(int(x) for x in b.lq[q]), []).append(q)
    for ls, qs in by_cls.items():
        s = inputs.subset(b, qs)
        o = oracle.eri_md4(ls, s.centers, s.exps, s.coefs, s.nprim)
        for i, q in enumerate(qs):
            res[q] = o[i]
    return res


def check(g_flat, offsets, b, idx):
    o = oracle_blocks(b, idx)
    for q in idx:
        ref = o[q]
        g = g_flat[offsets[q]:offsets[q] + ref.size].reshape(ref.shape)
        scale = max(np.abs(ref).max(), ZERO_SCALE)
        assert np.isfinite(g).all(), q
        assert np.abs(g - ref).max() <= TOL * scale, (q, tuple(b.lq[q]), np.abs(g - ref).max() / scale)


def test_plan_low_l_mixed_against_oracle(torch):
    b = mixed(60, 21, (0, 1, 2), 3)
    p = eri4.Plan(b.lq, b.nprim, b.kmax)
    off = p.offsets()
    sizes = np.array([eri4.quartet_size(*b.lq[q]) for q in range(b.nq)])
    assert off[0] == 0 and np.array_equal(off[1:], np.cumsum(sizes)[:-1]) and p.output_size == sizes.sum()
    out = p.execute(dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs))
    torch.cuda.synchronize()
    check(out.cpu().numpy(), off, b, range(b.nq))


def test_plan_high_l_mixed_against_oracle(torch):
    b = mixed(40, 22, (4, 5, 6), 2)
    p = eri4.Plan(b.lq, b.nprim, b.kmax)
    out = p.execute(dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs))
    torch.cuda.synchronize()
    idx = sorted({0, 39, *np.random.default_rng(0).choice(40, 8, replace=False).tolist()})
    check(out.cpu().numpy(), p.offsets(), b, idx)


def test_plan_matches_single_class_batches_bitwise(torch):
    b = mixed(50, 23, (4, 5, 6), 3)
    p = eri4.Plan(b.lq, b.nprim, b.kmax)
    C, E, Co = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs)
    out = p.execute(C, E, Co).cpu().numpy()
    off = p.offsets()
    for q in range(b.nq):
        s = inputs.subset(b, [q])
        g = eri4.batch(tuple(b.lq[q]), dev(torch, s.centers), dev(torch, s.exps), dev(torch, s.coefs),
                       dev(torch, s.nprim)).cpu().numpy()[0]
        assert np.array_equal(out[off[q]:off[q] + g.size].reshape(g.shape), g), q


def test_plan_graph_capture_replays(torch):
    b = mixed(30, 24, (4, 5), 2)
    p = eri4.Plan(b.lq, b.nprim, b.kmax)
    C, E, Co = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs)
    eager = p.execute(C, E, Co)
    torch.cuda.synchronize()
    ref = eager.cpu().numpy()
    out = torch.zeros_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        p.execute(C, E, Co, out=out, stream=s)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep
        # unrelated eager work between replays
        eri4.batch(tuple(b.lq[0]), C[:1].contiguous(), E[:1].contiguous(), Co[:1].contiguous(),
                   dev(torch, b.nprim[:1]))
        torch.cuda.synchronize()


def test_tile_choices_give_the_default_results(torch):
    """Every tile height and R layout that fits gives the integrals of the
    library's own choice (same arithmetic, other tiling), for classes that
    can use all three layouts."""
    b = mixed(24, 25, (4, 5), 3)
    C, E, Co = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs)
    ref = eri4.Plan(b.lq, b.nprim, b.kmax).execute(C, E, Co)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    classes = sorted({tuple(int(x) for x in r) for r in b.lq})
    for rows16, lay in ((1, "box"), (2, "box"), (4, "box"), (1, "box2"), (2, "box2"), (4, "box2"), (1, "slab"),
                        (2, "slab")):
        # two boxes fit up to total order 19 and 64-row tiles need kets with
        # lc+ld <= 9; other classes keep the default
        tiles = [{"l": c, "kq": (1, 4096), "rows16": rows16, "layout": lay} for c in classes
                 if (lay != "box2" or sum(c) <= 19) and (rows16 != 4 or c[2] + c[3] <= 9)]
        p = eri4.Plan(b.lq, b.nprim, b.kmax, tiles=tiles)
        g = p.execute(C, E, Co)
        torch.cuda.synchronize()
        g = g.cpu().numpy()
        scale = np.abs(ref).max()
        assert np.abs(g - ref).max() <= 1e-13 * scale, (rows16, lay, np.abs(g - ref).max() / scale)
    check(ref, p.offsets(), b, [0, 5, 11])


def test_tile_choice_that_does_not_fit_is_rejected(torch):
    lq = np.array([[6, 6, 6, 6]], np.int32)
    with pytest.raises(eri4.Eri4Error, match="does not fit"):
        eri4.Plan(lq, np.ones((1, 4), np.int32), 1, tiles=[{"l": (6, 6, 6, 6), "kq": (1, 1), "rows16": 2,
                                                            "layout": "box2"}])


def test_plan_over_l4_to_l7_sampled_against_oracle(torch):
    """A slice of the serving stream (classes in {4..7}^4, K=3 per shell): every
    integral finite, and the oracle on the quartets with the smallest total l
    plus two random ones of total l <= 18."""
    b = inputs.stream_batch(nq=200, seed=2106)
    p = eri4.Plan(b.lq, b.nprim, b.kmax)
    g = p.execute(dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    assert np.isfinite(g).all()
    tot = b.lq.sum(axis=1)
    small = np.flatnonzero(tot <= 18)
    idx = sorted({*np.argsort(tot, kind="stable")[:3].tolist(),
                  *np.random.default_rng(5).choice(small, 2, replace=False).tolist()})
    check(g, p.offsets(), b, idx)


def test_empty_plan(torch):
    p = eri4.Plan(np.zeros((0, 4), np.int32), np.zeros((0, 4), np.int32), 1)
    assert p.output_size == 0
    z = torch.zeros(0, 4, 3, dtype=torch.float64, device="cuda")
    p.execute(z, torch.zeros(0, 4, 1, dtype=torch.float64, device="cuda"),
              torch.zeros(0, 4, 1, dtype=torch.float64, device="cuda"),
              out=torch.zeros(1, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()


def test_tile_table_file_gives_the_plan_of_its_entries(torch, tmp_path):
    """eri4_plan_create_tunefile reads the committed table and builds the plan
    its entries give through eri4_plan_create_tuned (same bits); tables for
    another architecture, malformed lines and missing files are refused."""
    b = mixed(40, 26, (4, 5, 6), 3)
    C, E, Co = dev(torch, b.centers), dev(torch, b.exps), dev(torch, b.coefs)
    via_file = eri4.Plan(b.lq, b.nprim, b.kmax, tune_file=eri4.TUNE_FILE).execute(C, E, Co)
    via_list = eri4.Plan(b.lq, b.nprim, b.kmax, tiles=eri4.read_tile_table(eri4.TUNE_FILE)).execute(C, E, Co)
    torch.cuda.synchronize()
    assert torch.equal(via_file, via_list)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    with open(eri4.TUNE_FILE) as f:
        assert f"arch {arch}\n" in f.read()
    bad = {"other_arch.txt": "arch gfx000\n4 4 4 4 1 1 2 box\n",
           "no_arch.txt": "4 4 4 4 1 1 2 box\n",
           "bad_line.txt": f"arch {arch}\n4 4 4 4 1 1 2\n",
           "bad_layout.txt": f"arch {arch}\n4 4 4 4 1 1 2 cube\n"}
    for name, text in bad.items():
        p = tmp_path / name
        p.write_text(text)
        with pytest.raises(eri4.Eri4Error, match="tile table"):
            eri4.Plan(b.lq, b.nprim, b.kmax, tune_file=str(p))
    with pytest.raises(eri4.Eri4Error, match="cannot open"):
        eri4.Plan(b.lq, b.nprim, b.kmax, tune_file=str(tmp_path / "missing.txt"))
