"""Joins on several key columns (packed into one 64-bit word on the device)
against the oracle, which compares the key tuples column by column: NULL in
any key column matches nothing, a probe value outside the build column's type
range matches nothing, duplicates give one pair per matching build row."""
import numpy as np
import pytest

import oracle
from tests.helpers import tbl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def check(gq, ctx, build, bkeys, bpreds, probe, pkeys, ppreds):
    bd, pd_ = gq.to_device(build), gq.to_device(probe)
    jt = ctx.join_build(bd, bkeys, bpreds)
    _, _, cnt0 = ctx.join_probe(jt, pd_, pkeys, ppreds, capacity=0)
    ctx.sync_status()
    cap = int(cnt0.item())
    pi, bi, cnt = ctx.join_probe(jt, pd_, pkeys, ppreds, capacity=cap)
    assert ctx.sync_status() == 0
    n = int(cnt.item())
    epi, ebi = oracle.join(build, bkeys, bpreds, probe, pkeys, ppreds)
    assert n == len(epi) and n > 0
    assert np.array_equal(pi[:n].cpu().numpy(), epi) and np.array_equal(bi[:n].cpu().numpy(), ebi)
    jt.free()


@pytest.mark.parametrize("nb", [20_011, (1 << 20) + 777])
def test_two_int32_keys_nulls_duplicates(gq, ctx, nb):
    # Small builds take the hash index, builds of 2^20 rows or more the
    # partitioned table (index built from it on first probe).
    rng = np.random.default_rng(nb)
    npr = 2 * nb + 5
    a = rng.integers(-300, 300, nb).astype(np.int32)
    b = rng.integers(-2**31, 2**31 - 1, nb, dtype=np.int64).astype(np.int32) % 1000
    build = tbl(a=(a, rng.random(nb) > 0.05), b=(b.astype(np.int32), rng.random(nb) > 0.05),
                d=rng.integers(0, 10, nb).astype(np.int8))
    # Probe keys drawn from the build's tuples (matches) and fresh ones.
    pick = rng.integers(0, nb, npr)
    pa = np.where(rng.random(npr) < 0.7, a[pick], rng.integers(-300, 300, npr)).astype(np.int32)
    pb = np.where(rng.random(npr) < 0.7, b[pick], rng.integers(0, 1000, npr)).astype(np.int32)
    probe = tbl(a=(pa, rng.random(npr) > 0.05), b=(pb, rng.random(npr) > 0.05),
                d=rng.integers(0, 10, npr).astype(np.int16))
    check(gq, ctx, build, [0, 1], [("range", 2, 0, 7)], probe, [0, 1], [("ne", 2, 3)])


def test_three_keys_mixed_widths_and_wider_probe_types(gq, ctx):
    # Build keys int16, int8, int32 (56 bits); the probe carries them as
    # int64, int32, int64 with values outside the build types' ranges, which
    # must match nothing (no wrap-around onto a build value).
    rng = np.random.default_rng(7)
    nb, npr = 50_003, 120_007
    k1 = rng.integers(-2**15, 2**15, nb).astype(np.int16)
    k2 = rng.integers(-128, 128, nb).astype(np.int8)
    k3 = rng.integers(-5, 5, nb).astype(np.int32)
    build = tbl(x=k1, y=(k2, rng.random(nb) > 0.02), z=k3)
    pick = rng.integers(0, nb, npr)
    p1 = k1[pick].astype(np.int64)
    p1 = np.where(rng.random(npr) < 0.1, p1 + (1 << 16), p1)      # out of int16 range, same low bits
    p2 = k2[pick].astype(np.int32)
    p2 = np.where(rng.random(npr) < 0.1, p2 - 256, p2)             # out of int8 range, same low bits
    p3 = k3[pick].astype(np.int64)
    p3 = np.where(rng.random(npr) < 0.1, p3 + (1 << 32), p3)      # out of int32 range, same low bits
    probe = tbl(p1=p1, p2=(p2, rng.random(npr) > 0.02), p3=p3)
    check(gq, ctx, build, [0, 1, 2], [], probe, [0, 1, 2], [])


def test_composite_key_limits(gq, ctx):
    rng = np.random.default_rng(3)
    t = gq.to_device(tbl(a=rng.integers(0, 9, 1000), b=rng.integers(0, 9, 1000).astype(np.int32)))
    # int64 + int32 needs 96 bits: not packable.
    with pytest.raises(gq.GqError) as e:
        ctx.join_build(t, [0, 1])
    assert e.value.code == gq.GQ_ERR_UNSUPPORTED
    u = gq.to_device(tbl(a=rng.integers(0, 9, 1000).astype(np.int32), b=rng.integers(0, 9, 1000).astype(np.int32)))
    jt = ctx.join_build(u, [0, 1])
    # The probe names as many key columns as the build.
    with pytest.raises(gq.GqError) as e:
        ctx.join_probe(jt, u, [0])
    assert e.value.code == gq.GQ_ERR_INVALID
    # The fused pipelines group by the one probe key: single-key tables only.
    with pytest.raises(gq.GqError) as e:
        ctx.pipeline(u, [], [0], [("count*",)], join=jt, probe_key=0)
    assert e.value.code == gq.GQ_ERR_UNSUPPORTED
    assert ctx.sync_status() == 0
    jt.free()
