"""CPU oracle (test infrastructure only): FP64 brute-force nonbonded sums and plain
NumPy binning / exclusion-window references.  Never imported by the GPU library."""
