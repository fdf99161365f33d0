"""FP64 CPU oracle -- test infrastructure only (tests/, smoke(), bench.py's cpu_baseline)."""
