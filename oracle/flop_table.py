"""Writes ``flop_per_pair.json``: the FLOP per ordered pair of every pass,
counted by the oracle on its own per-pair code (``oracle.flops``).

Test infrastructure: the benchmark reads the table as the reference count of
each pass's algorithmic work.  Run ``python -m oracle.flop_table`` after any
change to the oracle's arithmetic; a CPU test fails while the file is stale.
"""

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "flop_per_pair.json")


def table():
    import oracle

    return {
        "flop_per_pair": oracle.flops(),
        "rules": "counted by oracle.flops(): operations of the oracle's per-pair code on values that "
                 "combine two particles (per-particle work hoisted), common subexpressions once, "
                 "constants folded; add/sub/mul/div/sqrt = 1 FLOP (multiply-add = 2), negation free; "
                 "adjoint passes = reverse-mode derivative of the pair term with respect to the lane "
                 "particle's inputs",
    }


def main():
    with open(TABLE, "w") as f:
        json.dump(table(), f, indent=1, sort_keys=True)
        f.write("\n")
    print(TABLE)


if __name__ == "__main__":
    main()
