"""Filter variants and the autotuner: every variant of every bucket is
bit-exact against the oracle; mt_autotune times the variants of the buckets
that hold pairs and keeps the fastest; the selection survives a JSON round
trip and a file from another architecture is refused."""
import json

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2311_02029_amd as mt_
    yield mt_
    mt_.tune_reset()


@pytest.fixture(scope="module")
def pairs(mt):
    """Pairs that populate every bucket: E <= 7 / 15 / 31, the four long bins
    (up to 20 kbp reads) and the general kernel (30 kbp)."""
    rnd = np.random.default_rng(31)
    gen = synth.make_genomes(rnd, 2, 150_000, 0.5)
    lens = np.array([150, 280, 900, 2500, 6000, 10_000, 20_000, 30_000, 75])
    reads, origin = synth.make_reads(rnd, gen, lens, 0.02, 0.02)
    pr, pg, pd, pe = [], [], [], []
    for i in range(reads.n):
        for E in (0, 5, 12, 25, 40, 130, 500, 1500):
            for shift in (0, -3, 17):
                pr.append(i)
                pg.append(origin[i, 0])
                pd.append(origin[i, 1] + shift)
                pe.append(E)
    pr, pg = np.array(pr, np.uint32), np.array(pg, np.uint32)
    pd, pe = np.array(pd, np.int64), np.array(pe, np.uint16)
    ga = gen.ascii()
    oap, oac = oracle.Index(ga, 15, 10).filter_pairs(reads, pr, pg, pd, pe)
    return dict(ga=ga, reads=reads, pr=pr, pg=pg, pd=pd, pe=pe, oap=oap, oac=oac)


def _run(mt, ix, p):
    import torch
    ap, ac = ix.filter_pairs(mt.to_device(p["reads"]), torch.from_numpy(p["pr"].view(np.int32)).cuda(),
                             torch.from_numpy(p["pg"].view(np.int32)).cuda(), torch.from_numpy(p["pd"]).cuda(),
                             torch.from_numpy(p["pe"].view(np.int16)).cuda())
    return ap.cpu().numpy().view(np.uint16), ac.cpu().numpy()


def test_every_variant_bit_exact(mt, pairs):
    ix = mt.Index(pairs["ga"], 15, 10)
    info = mt.tune_info()
    assert [b["name"] for b in info] == ["E<=7", "E<=15", "E<=31", "long<=96", "long<=192", "long<=384",
                                         "long<=768", "general"]
    tried = 0
    for b in info:
        for v, name in enumerate(b["variants"]):
            mt.tune_reset()
            try:
                mt.tune_set(b["bucket"], v)
            except mt.MTError as e:  # its LDS does not fit a workgroup
                assert e.status == mt._abi.MT_EINVAL and name.startswith("lds_w")
                continue
            ap, ac = _run(mt, ix, pairs)
            assert np.array_equal(ap, pairs["oap"]), (b["name"], name, np.flatnonzero(ap != pairs["oap"])[:10])
            assert np.array_equal(ac, pairs["oac"]), (b["name"], name)
            tried += 1
    mt.tune_reset()
    assert tried >= 20
    with pytest.raises(mt.MTError):
        mt.tune_set(0, 7)
    with pytest.raises(mt.MTError):
        mt.tune_set(8, 0)


def test_autotune_selects_fastest_and_round_trips(mt, pairs, tmp_path):
    rnd = np.random.default_rng(32)
    gen = synth.make_genomes(rnd, 3, 200_000, 0.5)
    lens = np.concatenate([rnd.integers(75, 301, 3000), rnd.integers(1000, 10_001, 60)])
    reads, _ = synth.make_reads(rnd, gen, lens, 0.01, 0.01)
    ga = gen.ascii()
    ix = mt.Index(ga, 15, 10)
    dr = mt.to_device(reads)
    q = dict(min_hits=3, top_n=3, e_mode=mt.MT_E_CEIL_PERMILLE, e_value=50)
    mt.tune_reset()
    before = ix.classify(dr, mode=mt.MT_MODE_PER_STAGE, **q).to_host()
    info = ix.autotune(dr, reps=2, **q)
    timed = [b for b in info if b["pairs"] > 0]
    assert {b["name"] for b in timed} >= {"E<=7", "E<=15", "long<=96"}
    for b in timed:
        assert b["ms"], b
        assert b["current"] == min(b["ms"], key=b["ms"].get), b
    after = ix.classify(dr, mode=mt.MT_MODE_PER_STAGE, **q).to_host()
    for f in ("cand_offsets", "genome", "diag", "hits", "approx", "accept", "unique", "multi"):
        assert np.array_equal(before[f], after[f]), f
    ref = oracle.Index(ga, 15, 10).classify(reads, 3, 3, 1, 50)
    for f in ("cand_offsets", "genome", "diag", "hits", "approx", "accept"):
        assert np.array_equal(np.asarray(after[f]), np.asarray(ref[f]).astype(after[f].dtype)), f

    path = str(tmp_path / "tune.json")
    mt.tune_save(path)
    sel = {b["name"]: b["current"] for b in mt.tune_info()}
    rec = json.load(open(path))
    assert rec["arch"].startswith("gfx") and rec["buckets"] == sel
    mt.tune_reset()
    mt.tune_load(path)
    assert {b["name"]: b["current"] for b in mt.tune_info()} == sel
    rec["arch"] = "gfx000"
    bad = tmp_path / "other.json"
    bad.write_text(json.dumps(rec))
    with pytest.raises(mt.MTError) as e:
        mt.tune_load(str(bad))
    assert e.value.status == mt._abi.MT_EINVAL
    mt.tune_reset()
