"""Run the oracle pin sets against one compiled oracle library, in its own process.

Usage: python -m tests.run_pins <path-to-oracle.so>
Exit status 0 when every pin holds, 1 when a pin fails. A crash of a mutated
oracle also ends the process with a non-zero status, which counts as caught.
"""
import sys

import oracle
from tests import pins


def main(path: str) -> int:
    lib = oracle.load_library(path)
    for pin in (lambda: pins.pin_paper_examples(lib), lambda: pins.pin_closed_forms(lib),
                lambda: pins.pin_exhaustive(lib, 4), lambda: pins.pin_random_digraphs(lib, 20),
                lambda: pins.pin_min_parents(lib), lambda: pins.pin_checkers_directed_counterexample(lib),
                lambda: pins.pin_checkers_exhaustive(lib), lambda: pins.pin_checkers_planted(lib)):
        fails = pin()
        if fails:
            print("PIN FAILED:", fails[0])
            return 1
    print("ALL PINS HOLD")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1]))
