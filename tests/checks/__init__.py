"""Independent checkers used to pin the oracle: dense linear algebra, brute
force and closed forms written from the mathematics, never from the oracle."""
