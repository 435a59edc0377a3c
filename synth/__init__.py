"""Seeded synthetic inputs and error metrics shared by tests and benchmark.

Holds no step of the MDS method, so it can feed both the FP64 oracle and the
HIP library without coupling them."""
