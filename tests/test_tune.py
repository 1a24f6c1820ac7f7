"""The launch-shape tuning table (host side of libhmc; no GPU needed)."""
import os

import pytest

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1212_0785_amd", "libhmc.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhmc.so not built")


@pytest.fixture(scope="module")
def H():
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def test_table_load_query_and_save(H, tmp_path):
    if os.environ.get("HMC_DSLASH_SPLIT") or os.environ.get("HMC_GFORCE_PLANES"):
        pytest.skip("environment overrides the table")
    src = tmp_path / "tune.txt"
    src.write_text("# comment line\n"
                   "dslash 6 2 2 10 0 2 12.5\n"
                   "dslash 6 2 2 10 1 4 7.0\n"
                   "gauge_force 6 2 2 10 0 1 90.0\n"
                   "dslash 6 2 2 10 0 3 1.0\n"       # invalid shape: ignored
                   "nonsense 1 2 3\n"
                   "dslash 6 2 2 10 9 1 1.0\n")      # invalid precision: ignored
    assert H.hmc_tune_load(str(src)) == 3
    assert H.hmc_tune_query((6, 2, 2, 10), H.TUNE_DSLASH, H.F64) == (2, True)
    assert H.hmc_tune_query((6, 2, 2, 10), H.TUNE_DSLASH, H.F32) == (4, True)
    assert H.hmc_tune_query((6, 2, 2, 10), H.TUNE_GAUGE_FORCE) == (1, True)
    # untuned entries follow the built-in rule (small volume: F64 one site
    # per work-item, FP32 arithmetic 4-way split, staple force four
    # directions per block)
    assert H.hmc_tune_query((6, 2, 2, 10), H.TUNE_DSLASH, H.F16) == (4, False)
    assert H.hmc_tune_query((4, 4, 4, 6), H.TUNE_DSLASH, H.F64) == (1, False)
    assert H.hmc_tune_query((4, 4, 4, 6), H.TUNE_GAUGE_FORCE) == (2, False)
    # save merges with what the file already holds
    dst = tmp_path / "out.txt"
    dst.write_text("dslash 2 2 2 2 0 4 3.0\n")
    n = H.hmc_tune_save(str(dst))
    lines = [ln.split() for ln in dst.read_text().splitlines() if ln and not ln.startswith("#")]
    assert n == len(lines) >= 4
    assert ["dslash", "2", "2", "2", "2", "0", "4", "3.000"] in lines
    assert ["dslash", "6", "2", "2", "10", "1", "4", "7.000"] in lines
    with pytest.raises(H.HmcError):
        H.hmc_tune_query((5, 2, 2, 10), H.TUNE_DSLASH, H.F64)  # odd extent
    with pytest.raises(H.HmcError):
        H.hmc_tune_load(str(tmp_path / "missing.txt"))


def test_link_form_entries(H, tmp_path):
    if os.environ.get("HMC_LINK_FORM"):
        pytest.skip("environment overrides the table")
    src = tmp_path / "links.txt"
    src.write_text("dslash_links 6 4 2 10 0 10 80.0\n"
                   "dslash_links 6 4 2 10 1 12 40.0\n"
                   "gauge_force_links 6 4 2 10 0 12 90.0\n"
                   "dslash_links 6 4 2 10 2 18 1.0\n"    # the full form is not a tunable choice
                   "gauge_force_links 6 4 2 10 0 11 1.0\n")
    assert H.hmc_tune_load(str(src)) == 3
    assert H.hmc_tune_query((6, 4, 2, 10), H.TUNE_DSLASH_LINKS, H.F64) == (H.LINK_ROWCOL, True)
    assert H.hmc_tune_query((6, 4, 2, 10), H.TUNE_DSLASH_LINKS, H.F32) == (H.LINK_ROWS2, True)
    assert H.hmc_tune_query((6, 4, 2, 10), H.TUNE_GAUGE_FORCE_LINKS) == (H.LINK_ROWS2, True)
    # built-in rule: two rows for the hop kernels below 2^20 half-lattice
    # sites, row 0 + column 2 above it and for the staple kernels
    assert H.hmc_tune_query((6, 4, 2, 10), H.TUNE_DSLASH_LINKS, H.F16) == (H.LINK_ROWS2, False)
    assert H.hmc_tune_query((48, 48, 48, 96), H.TUNE_DSLASH_LINKS, H.F64)[0] in (H.LINK_ROWCOL, H.LINK_ROWS2)
    assert H.hmc_tune_query((64, 64, 64, 64), H.TUNE_DSLASH_LINKS, H.F64) == (H.LINK_ROWCOL, False)
    assert H.hmc_tune_query((4, 4, 4, 6), H.TUNE_GAUGE_FORCE_LINKS) == (H.LINK_ROWCOL, False)
    with pytest.raises(H.HmcError):
        H.hmc_tune_query((6, 4, 2, 10), 7, H.F64)  # no such kind


def test_stream_entries(H, tmp_path):
    if os.environ.get("HMC_LINK_STREAM"):
        pytest.skip("environment overrides the table")
    src = tmp_path / "stream.txt"
    src.write_text("dslash_stream 6 4 4 10 0 1 80.0\n"
                   "dslash_stream 6 4 4 10 1 0 40.0\n"
                   "dslash_stream 6 4 4 10 2 2 1.0\n")   # not 0/1: ignored
    assert H.hmc_tune_load(str(src)) == 2
    assert H.hmc_tune_query((6, 4, 4, 10), H.TUNE_DSLASH_STREAM, H.F64) == (1, True)
    assert H.hmc_tune_query((6, 4, 4, 10), H.TUNE_DSLASH_STREAM, H.F32) == (0, True)
    # rule: streaming from 2^20 half-lattice sites
    assert H.hmc_tune_query((6, 4, 4, 10), H.TUNE_DSLASH_STREAM, H.F16) == (0, False)
    assert H.hmc_tune_query((64, 64, 64, 64), H.TUNE_DSLASH_STREAM, H.BF16) == (1, False)


def test_order_entries_need_an_admissible_lattice(H, tmp_path):
    if os.environ.get("HMC_DSLASH_ORDER"):
        pytest.skip("environment overrides the table")
    src = tmp_path / "order.txt"
    src.write_text("dslash_order 16 8 4 8 0 1 1.0\n"     # admissible
                   "dslash_order 6 4 4 10 0 1 1.0\n"     # 6*4*4/2 = 48 sites per t-slice: not a multiple of 64
                   "dslash_order 48 16 4 8 0 3 1.0\n"    # 384 sites per z-plane = 6 chunks: y-blocks of 3
                   "dslash_order 48 16 4 8 1 4 1.0\n"    # 4 does not divide 6: whole z-planes
                   "dslash_order 48 16 4 8 2 65 1.0\n"   # beyond 64 chunks: ignored
                   "dslash_order 24 12 8 16 0 2 1.0\n")  # z-planes not whole chunks: the t-slice walk (1)
    assert H.hmc_tune_load(str(src)) == 5
    assert H.hmc_tune_query((16, 8, 4, 8), H.TUNE_DSLASH_ORDER, H.F64) == (1, True)
    assert H.hmc_tune_query((6, 4, 4, 10), H.TUNE_DSLASH_ORDER, H.F64) == (0, True)
    assert H.hmc_tune_query((16, 8, 4, 8), H.TUNE_DSLASH_ORDER, H.F32) == (0, False)
    assert H.hmc_tune_query((48, 16, 4, 8), H.TUNE_DSLASH_ORDER, H.F64) == (3, True)
    assert H.hmc_tune_query((48, 16, 4, 8), H.TUNE_DSLASH_ORDER, H.F32) == (1, True)
    assert H.hmc_tune_query((48, 16, 4, 8), H.TUNE_DSLASH_ORDER, H.F16) == (0, False)
    assert H.hmc_tune_query((24, 12, 8, 16), H.TUNE_DSLASH_ORDER, H.F64) == (1, True)


def test_occupancy_entries(H, tmp_path):
    if os.environ.get("HMC_DSLASH_OCC"):
        pytest.skip("environment overrides the table")
    src = tmp_path / "occ.txt"
    src.write_text("dslash_occupancy 48 16 4 8 0 0 1.0\n"
                   "dslash_occupancy 48 16 4 8 1 2 1.0\n"
                   "dslash_occupancy 48 16 4 8 2 1 1.0\n")  # not 0 / 2: ignored
    assert H.hmc_tune_load(str(src)) == 2
    assert H.hmc_tune_query((48, 16, 4, 8), H.TUNE_DSLASH_OCC, H.F64) == (0, True)
    assert H.hmc_tune_query((48, 16, 4, 8), H.TUNE_DSLASH_OCC, H.F32) == (2, True)
    assert H.hmc_tune_query((48, 16, 4, 8), H.TUNE_DSLASH_OCC, H.F16) == (2, False)  # rule: at most two
