"""Launch shapes of the expansion kernel for every tuning setting, checked on
the CPU against the kernel's limits (no device needed): the per-round change
mask fits 64 bits, a lane stages whole 16-byte units, the staging fits the
LDS a block may allocate, a lane's range is whole rounds, and the grid covers
the rows in whole XCD rounds."""
import itertools

import pytest

LDS_PER_BLOCK = 160 * 1024  # gfx950: LDS per compute unit, all of it addressable by one block


def _check(cfg, n_rows):
    assert cfg["stage"] in (2, 4, 8)
    assert cfg["change_bits"] == cfg["stage"] * cfg["kernel_tables"] <= 64
    assert cfg["seg_bytes"] % 16 == 0 and cfg["seg_bytes"] > 0
    assert cfg["tuples_per_lane"] % cfg["stage"] == 0 and cfg["tuples_per_lane"] >= cfg["stage"]
    assert 0 < cfg["lds_used"] <= cfg["lds_bytes"] <= LDS_PER_BLOCK
    assert cfg["lds_used"] >= 256 * cfg["seg_bytes"]
    assert cfg["blocks"] % 8 == 0 and cfg["blocks"] <= 2**31 - 1
    assert cfg["blocks"] * 256 * cfg["tuples_per_lane"] >= n_rows


ROWS = [1, 7, 4097, (1 << 20) + 3, 1 << 28, (1 << 31) + 5]


def test_row_id_launches_every_setting():
    from paper_2206_10435_amd import gj

    n_checked = 0
    for n, wb, stage, rounds, rows in itertools.product(range(1, 17), (4, 8), (2, 4, 8),
                                                         (0, 1, 3, 5, 7, 17, 1024), ROWS):
        cfg = gj.desum_launch_config(n, wb, 0, rows, gj.Tune(8, 8, rounds, stage))
        _check(cfg, rows)
        assert cfg["kernel_tables"] == (n if n <= 8 else 16)
        n_checked += 1
    assert n_checked == 16 * 2 * 3 * 7 * len(ROWS)


def test_value_launches_every_setting():
    from paper_2206_10435_amd import gj

    for n, nc, rounds, rows in itertools.product(range(1, 17), range(1, 17), (0, 1, 7), ROWS):
        cfg = gj.desum_launch_config(n, 4, nc, rows, gj.Tune(8, 8, rounds, 4))
        _check(cfg, rows)
        assert cfg["kernel_tables"] >= n


def test_tune_variants_of_the_parity_test():
    """The settings the GPU parity test sweeps (sort tiles, digit widths,
    rounds 1/3/17/5/1, stages 4/2/8/2/8) on its 4-table query and on every
    table count."""
    from paper_2206_10435_amd import gj

    for si, rb, dr, ds in [(8, 4, 1, 4), (16, 6, 3, 2), (8, 8, 17, 8), (16, 7, 5, 2), (16, 8, 1, 8)]:
        for n in range(1, 17):
            for wb in (4, 8):
                for rows in ROWS:
                    _check(gj.desum_launch_config(n, wb, 0, rows, gj.Tune(si, rb, dr, ds)), rows)


def test_unsupported_launches_refused():
    from paper_2206_10435_amd import gj

    for args in [(0, 8, 0, 10), (17, 8, 0, 10), (3, 2, 0, 10), (3, 8, 1, 10), (3, 4, 17, 10), (3, 8, 0, -1)]:
        with pytest.raises(gj.GJError):
            gj.desum_launch_config(*args)
