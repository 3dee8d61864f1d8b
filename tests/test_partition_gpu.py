"""gq_hash_partition on the GPU against the oracle, bit-exact (rows, order, offsets)."""
import numpy as np
import pytest

import oracle
from paper_2606_24647_amd import datagen as dg
from tests.helpers import assert_col_equal, random_table, tbl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gq():
    from paper_2606_24647_amd import gq as mod
    return mod


@pytest.fixture(scope="module")
def ctx(gq):
    return gq.Context()


def check_partition(gq, ctx, table, keys, P, seed=0):
    dev = gq.to_device(table)
    out, offs = ctx.hash_partition(dev, keys, P, seed)
    assert ctx.sync_status() == 0
    perm, eoff = oracle.partition(table, keys, P, seed)
    assert np.array_equal(offs.cpu().numpy(), eoff)
    got = gq.read_table(out, table.nrows)
    for j, c in enumerate(table.cols):
        ev = c.data[perm]
        eok = None if c.valid is None else c.valid[perm]
        assert_col_equal(got[j], ev, eok, f"col {j}")


@pytest.mark.parametrize("P", [1, 2, 3, 64, 256, 257, 1000, 1024])
def test_partition_P(gq, ctx, P):
    t = dg.batch_c3(123_457, nkeys=50_000, seed=P)
    check_partition(gq, ctx, t, [0], P)


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 4095, 4096, 4097, 9000])
def test_partition_sizes(gq, ctx, n):
    rng = np.random.default_rng(n)
    check_partition(gq, ctx, random_table(rng, n), [0], 64, seed=7)


def test_partition_nulls_multikey_seed(gq, ctx):
    rng = np.random.default_rng(2)
    t = random_table(rng, 50_001, null_frac=0.25)
    check_partition(gq, ctx, t, [3, 1], 256, seed=0xDEADBEEF12345678)


def test_partition_all_equal_keys(gq, ctx):
    t = tbl(k=np.full(40_000, 77, dtype=np.int64), v=np.arange(40_000, dtype=np.int32))
    check_partition(gq, ctx, t, [0], 256)


def test_partition_bad_nparts(gq, ctx):
    t = gq.to_device(tbl(k=np.arange(10, dtype=np.int64)))
    for P in (0, 1025):
        with pytest.raises(gq.GqError):
            ctx.hash_partition(t, [0], P)


@pytest.mark.parametrize("ncols", [4, 5, 12])
def test_partition_wide_rows(gq, ctx, ncols):
    # Rows of ncols int64 columns: 4 still fit the 4096-row staging of the
    # 1024-thread scatter, 5 and 12 take the 1024-row variant.
    rng = np.random.default_rng(ncols)
    n = 70_001
    cols = {f"c{j}": rng.integers(-10**12, 10**12, n) for j in range(ncols)}
    cols["c1"] = (cols["c1"], rng.random(n) > 0.2)
    check_partition(gq, ctx, tbl(**cols), [0, 1], 64, seed=3)
