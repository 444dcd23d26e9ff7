"""gj_summary_file_check on the host: a consistent stored summary is accepted
with its header read back, and every damaged copy (bad header, bad table
header, a section out of range, truncation, trailing bytes) is refused with
GJ_E_INVALID.  No device is used."""
import pytest

import store_file_cases as SF


def test_consistent_file_is_accepted(tmp_path):
    from paper_2206_10435_amd import gj

    for with_rows in (True, False):
        p = tmp_path / f"good{int(with_rows)}.gjs"
        b = SF.build(with_rows=with_rows)
        p.write_bytes(b)
        info = gj.summary_file_check(str(p))
        assert info == {"n_tables": 2, "projected": False, "with_rows": with_rows, "join_size": 6,
                        "entries": [2, 2], "rows": [3, 2], "bytes": len(b)}


@pytest.mark.parametrize("case", SF.damaged(), ids=lambda c: c[0])
def test_damaged_file_is_refused(tmp_path, case):
    from paper_2206_10435_amd import gj

    reason, data = case
    p = tmp_path / "bad.gjs"
    p.write_bytes(data)
    with pytest.raises(gj.GJError) as ei:
        gj.summary_file_check(str(p))
    assert ei.value.status == gj.GJ_E_INVALID, reason


def test_missing_file_is_refused(tmp_path):
    from paper_2206_10435_amd import gj

    with pytest.raises(gj.GJError) as ei:
        gj.summary_file_check(str(tmp_path / "absent.gjs"))
    assert ei.value.status == gj.GJ_E_INVALID and "cannot open" in str(ei.value)
