"""Run inside a process that preloads the address sanitizer: the runtime's
host-only entry points (graph validation, the junction tree, launch shapes,
the stored-summary file check) from a sanitizer build of the library whose
path is argv[1]; argv[2] is a scratch directory.  Any out-of-bounds access,
use after free or undefined behaviour aborts the process."""
import itertools
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import store_file_cases as SF  # noqa: E402
from paper_2206_10435_amd import gj  # noqa: E402


def expect_error(fn, *a):
    try:
        fn(*a)
    except gj.GJError as e:
        return e.status
    raise AssertionError(f"{fn.__name__}{a} did not fail")


def main():
    gj.load_library(sys.argv[1])
    tmp = sys.argv[2]
    # graph validation: good trees, then broken ones
    gj.validate([5, 6, 7], [2, 2, 2], [-1, 0, 1], [0, 0, 0], [0, 1, 1])
    gj.validate([5] * 16, [8] * 16, [-1] + list(range(15)), [0] * 16, [7] * 16)
    for args in [([5, 6], [2, 2], [-1, 1], [0, 0], [0, 1]),      # parent not earlier
                 ([5, 6], [2, 2], [-1, 0], [0, 2], [0, 1]),      # separator column out of range
                 ([5, 6], [2, 2], [-1, 0], [0, 0], [0, 2]),      # parent column out of range
                 ([5, 6], [0, 2], [-1, 0], [0, 0], [0, 1]),      # no key column
                 ([5, 6], [9, 2], [-1, 0], [0, 0], [0, 1]),      # too many key columns
                 ([5] * 17, [2] * 17, [-1] + list(range(16)), [0] * 17, [1] * 17),  # too many tables
                 ([-1, 6], [2, 2], [-1, 0], [0, 0], [0, 1])]:    # negative row count
        expect_error(gj.validate, *args)
    # junction trees: acyclic, triangle, 4-cycle, clique, disconnected, bad ids
    for attrs in ([[0, 1], [1, 2], [2, 3]], [[0, 1], [1, 2], [0, 2]], [[0, 1], [1, 2], [2, 3], [3, 0]],
                  [[0, 1, 2, 3], [1, 2], [3, 4, 5, 6, 7, 8, 9, 10]], [[i, i + 1] for i in range(15)],
                  [[0, 9], [9, 4], [4, 0], [4, 7], [7, 0]]):
        jt = gj.junction_tree(attrs)
        assert len(jt["table_clique"]) == len(attrs)
    expect_error(gj.junction_tree, [[0, 1], [2, 3]])
    expect_error(gj.junction_tree, [[0, -1], [1, 2]])
    expect_error(gj.junction_tree, [[i, i + 1] for i in range(0, 140, 2)][:16])
    # launch shapes of the expansion kernel
    for n, wb, stage, rounds, rows in itertools.product(range(1, 17), (4, 8), (2, 4, 8), (0, 1, 7, 1024),
                                                         (1, 4097, (1 << 31) + 5)):
        gj.desum_launch_config(n, wb, 0, rows, gj.Tune(8, 8, rounds, stage))
    for n, nc in itertools.product(range(1, 17), range(1, 17)):
        gj.desum_launch_config(n, 4, nc, 1 << 28, gj.Tune(8, 8, 0, 4))
    expect_error(gj.desum_launch_config, 0, 8, 0, 10)
    expect_error(gj.desum_launch_config, 4, 2, 0, 10)
    expect_error(gj.desum_launch_config, 17, 4, 0, 10)
    # stored summaries: the consistent file, then every damaged one
    p = os.path.join(tmp, "s.gjs")
    for with_rows in (True, False):
        with open(p, "wb") as f:
            f.write(SF.build(with_rows=with_rows))
        assert gj.summary_file_check(p)["n_tables"] == 2
    for reason, data in SF.damaged():
        with open(p, "wb") as f:
            f.write(data)
        assert expect_error(gj.summary_file_check, p) == gj.GJ_E_INVALID, reason
    expect_error(gj.summary_file_check, os.path.join(tmp, "absent.gjs"))
    print("sanitized runtime host paths ok", flush=True)


if __name__ == "__main__":
    main()
