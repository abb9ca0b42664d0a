"""Storage accounting of matrices and factors (Sections 3.4, 4.1, 4.2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.4: the memory a dense matrix needs follows exactly from its shape and
scalar size.  The experiments quote such counts: the rank-50 factors of a
512 x 512 image hold 51,250 values, 102,500 bytes in half and 410,000 bytes in
double precision (Section 4.2.2); the two sparse test matrices would take more
than 15 TB and roughly 225 TB stored dense (Section 4.1).

Parity pins: tests/golden/paper_storage.json (those printed figures).
"""

SCALAR_BYTES = {"f16": 2, "bf16": 2, "f32": 4, "f64": 8, "fp8": 1}


def factor_values(m, n, k):
    """Values in U (m x k), the k singular values and V (n x k)."""
    return m * k + k + n * k


def dense_bytes(m, n, dtype):
    return m * n * SCALAR_BYTES[dtype]


def values_bytes(count, dtype):
    return count * SCALAR_BYTES[dtype]
