"""TEST INFRASTRUCTURE ONLY: the serial FP64 CPU oracle (see oracle.py)."""
