"""Host-side tests of the autotuner and cost-model boundary (no GPU): the
candidate set and features follow the rule the header documents, the
library's median and tie rule equal the oracle's, a malformed timing
database is refused, and a missing, corrupt or foreign cost-model file makes
the choice fall back to the tuner and then to the defaults."""
import math
import struct

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import tuner as OT
from paper_2110_14340_amd import jacc, tuner

BLOCKS = [(64, 1), (128, 1), (256, 1), (512, 1), (64, 4), (128, 2), (256, 2), (256, 4)]


def documented_candidates(shape, ks):
    """The candidate order written out from the header's description."""
    out = []
    even = shape[-1] % 2 == 0
    for K in ks:
        if K > shape[0] - 2:
            continue
        for bx, by in BLOCKS:
            for rows in ([1, 4] if len(shape) == 3 else [1]):
                if rows > 1 and bx * by > 256:
                    continue
                for tile in (1, 4, 16, 64):
                    for vec in (1, 2):
                        if vec == 2 and not even:
                            continue
                        out.append({"bx": bx, "by": by, "tile": tile, "vec": vec, "persistent": 0, "rows": rows,
                                    "K": K})
        for tile in (1, 4, 16):
            for vec in (1, 2):
                if vec == 2 and not even:
                    continue
                out.append({"bx": 256, "by": 1, "tile": tile, "vec": vec, "persistent": 1, "rows": 1, "K": K})
    return out


@pytest.mark.parametrize("shape,ks", [((64, 130), [1, 2, 4, 8]), ((33, 67), [1, 2]), ((5, 64), [1, 2, 4, 8]),
                                      ((40, 34, 66), [1, 2, 4, 8]), ((9, 9, 9), [8, 1])])
def test_candidates_follow_the_documented_order(shape, ks):
    assert jacc.candidates(shape, ks) == documented_candidates(shape, ks)


def test_candidate_counts_and_errors():
    assert len(jacc.candidates((100, 100), [1, 2, 4, 8])) == 4 * (64 + 6)
    assert len(jacc.candidates((100, 100, 100), [1, 2, 4, 8])) == 4 * (104 + 6)
    with pytest.raises(jacc.JaccError):
        jacc.candidates((100,), [1])
    with pytest.raises(jacc.JaccError):
        jacc.candidates((100, 100), [0])


@pytest.mark.parametrize("shape", [(64, 130), (4096, 77), (34, 40, 66), (512, 32, 511)])
def test_features_follow_the_documented_definition(shape):
    for c in jacc.candidates(shape, [1, 2, 8])[::7]:
        f = jacc.features(shape, c)
        dims = list(shape) + [1] * (3 - len(shape))
        cells = float(np.prod([d - 2 for d in shape]))
        bx, by = (256, 1) if c["persistent"] else (c["bx"], c["by"])
        if len(shape) == 2:
            wg = math.ceil((shape[1] - 2) / (bx * c["vec"])) * math.ceil((shape[0] - 2) / (by * c["tile"]))
        else:
            wg = (math.ceil((shape[2] - 2) / (bx * c["vec"])) * math.ceil((shape[1] - 2) / (by * c["rows"]))
                  * math.ceil((shape[0] - 2) / c["tile"]))
        ref = [float(len(shape) == 3), math.log2(dims[0]), math.log2(dims[1]), math.log2(dims[2]), math.log2(cells),
               math.log2(c["bx"]), math.log2(c["by"]), math.log2(c["tile"]), c["vec"], math.log2(c["K"]),
               c["persistent"], math.log2(wg), math.log2(c["rows"])]
        assert np.allclose(f, np.float32(ref), rtol=1e-6, atol=1e-6), (c, f, ref)


@settings(max_examples=300, deadline=None)
@given(st.lists(st.lists(st.floats(1e-6, 1e3, allow_nan=False), min_size=1, max_size=12), min_size=1, max_size=30))
def test_library_selection_rule_equals_oracle(samples):
    meds = [jacc.median(s) for s in samples]
    assert meds == [OT.median(s) for s in samples]
    assert tuner.select(meds) == OT.select(samples)


def test_selection_ties_go_to_the_lowest_index():
    assert jacc.argmin([3.0, 1.0, 2.0, 1.0]) == 1
    assert jacc.median([4, 1, 3, 2]) == 2.5
    assert OT.select([[2.0], [1.0, 1.0], [1.0]]) == tuner.select([2.0, 1.0, 1.0]) == 1


# ------------------------------------------------------------------ files and fallbacks
def dry_ctx():
    return jacc.Context(2, flags=jacc.INIT_DRYRUN)


def _arrays(c, shape=(40, 66)):
    u = np.zeros(shape)
    v = np.zeros(shape)
    c.enter(u, halo=(1, 1))
    c.enter(v, halo=(1, 1))
    return u, v


def test_malformed_timing_database_is_refused_and_kept(tmp_path):
    c = dry_ctx()
    u, v = _arrays(c)
    db = tmp_path / "t.db"
    db.write_text("1 40 66 0 1 64 1 1 1 0 1 2 0.1 0.2\n")  # an entry before any section
    with pytest.raises(jacc.JaccError) as e:
        c.tune(u, v, ks=[1], db_path=str(db))
    assert e.value.status == jacc.ERR_INVALID and "entry before any section" in str(e.value)
    db.write_text("@ k\n1 40 66 0 1 64 1 1 1 0 1 3 0.1 0.2\n")  # three samples announced, two given
    with pytest.raises(jacc.JaccError) as e:
        c.tune(u, v, ks=[1], db_path=str(db))
    assert "bad sample" in str(e.value)
    assert db.read_text().startswith("@ k")  # never overwritten
    db.write_text("@ k\n1 40 66 0 1 64 1 1 1 0 1 2 0.1 0.2\n")  # well formed: the dry context then refuses timing
    with pytest.raises(jacc.JaccError) as e:
        c.tune(u, v, ks=[1], db_path=str(db))
    assert e.value.status == jacc.ERR_UNSUPPORTED
    c.close()


def _model_file(path, key, members=1, corrupt=False, F=13):
    P = jacc.lib().jacc_model_nparams(F)
    body = b"JACCCM01" + struct.pack("<I", len(key)) + key.encode() + struct.pack("<ii", F, members)
    body += np.zeros(F, np.float32).tobytes() + np.ones(F, np.float32).tobytes()
    body += np.zeros(members * P, np.float32).tobytes()
    h = 1469598103934665603
    for b in body:
        h = ((h ^ b) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    data = body + struct.pack("<Q", h)
    if corrupt:
        data = data[:40] + bytes([data[40] ^ 1]) + data[41:]
    path.write_bytes(data)


def test_model_file_checks(tmp_path):
    c = dry_ctx()
    key = c.build_key()
    assert key.startswith("dry|hip0|") and len(key.split("|")[2]) == 12
    good, bad, foreign, trunc = (tmp_path / n for n in ("good.bin", "bad.bin", "foreign.bin", "trunc.bin"))
    _model_file(good, key)
    _model_file(bad, key, corrupt=True)
    _model_file(foreign, "gfx942|hip1|000000000000")
    trunc.write_bytes(good.read_bytes()[:-9])
    assert c.model_load(str(tmp_path / "missing.bin"), raw=True) == jacc.ERR_INVALID
    assert "cannot open" in c.last_error()
    assert c.model_load(str(bad), raw=True) == jacc.ERR_INVALID
    assert "checksum" in c.last_error()
    assert c.model_load(str(trunc), raw=True) == jacc.ERR_INVALID
    assert c.model_load(str(foreign), raw=True) == jacc.ERR_INVALID
    assert "build key gfx942" in c.last_error()
    # a well-formed file passes every check; the dry context then has no device for it
    assert c.model_load(str(good), raw=True) == jacc.ERR_UNSUPPORTED
    assert c.model_pick((40, 66), [1], raw=True) == jacc.ERR_INVALID  # nothing attached
    c.close()


def test_choice_falls_back_from_a_corrupt_model_to_the_tuner_then_the_defaults(tmp_path):
    c = dry_ctx()
    u, v = _arrays(c)
    bad = tmp_path / "bad.bin"
    _model_file(bad, c.build_key(), corrupt=True)
    cand, src = c.choose(u, v, model_path=str(bad), ks=[1, 2])
    # the model is refused (checksum), the tuner cannot time in a dry-run
    # context, so the defaults at the arrays' K remain
    assert src == jacc.CHOICE_DEFAULT
    assert cand == {"bx": 0, "by": 0, "tile": 0, "vec": 0, "persistent": 0, "rows": 0, "K": 2}
    msg = c.last_error()
    assert "model:" in msg and "checksum" in msg and "tuner:" in msg and "needs the device" in msg
    cand, src = c.choose(u, v, tune=False)
    assert src == jacc.CHOICE_DEFAULT and cand["K"] == 2
    c.close()
