"""CPU oracle (test infrastructure).  See oracle.py."""
