"""The device generator reproduces the host generator bit for bit (input generation only)."""
import numpy as np
import pytest

from paper_2606_24647_amd import datagen as dg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def devgen():
    from paper_2606_24647_amd import devgen as mod
    return mod


def same(dev_table, host_table):
    for d, h in zip(dev_table.cols, host_table.cols):
        assert np.array_equal(d.data.cpu().numpy(), h.data)


def test_fact_c1(devgen):
    same(devgen.fact_c1(100_003, start=12_345), dg.fact_c1(100_003, start=12_345))


def test_fact_and_dim_c2(devgen):
    same(devgen.fact_c2(50_000, nkeys=7_777, start=999), dg.fact_c2(50_000, nkeys=7_777, start=999))
    same(devgen.dim_c2(123_457), dg.dim_c2(123_457))
    same(devgen.dim_c2(4_000_000, start=3_990_000), dg.dim_c2(4_000_000, start=3_990_000))


def test_batch_c3(devgen):
    same(devgen.batch_c3(77_777, nkeys=15_000_000, start=5), dg.batch_c3(77_777, nkeys=15_000_000, start=5))


def test_fragment(devgen):
    spec = dg.fragments_c4(16)
    for f in range(3):
        rows, card = int(spec.rows[f]), int(spec.card[f])
        same(devgen.fragment_c4(f, rows, card), dg.fragment_c4(f, rows, card))


def test_serving_tables(devgen):
    same(devgen.fact_c5(50_001, nkeys=10_000, start=77), dg.fact_c5(50_001, nkeys=10_000, start=77))
    same(devgen.dim_c5(30_000), dg.dim_c5(30_000))
