"""Work and traffic accounting for one gate-application pass.

A pass applies one (fused) k-qubit gate to all 2^(n-k) groups of an n-qubit
complex64 state (Sec. II-A, Eq. 4).  Per group the matrix-vector product costs
2^k complex rows, each with 2^k complex multiplies (6 flops) and 2^k - 1
complex adds (2 flops): 2^k (8 * 2^k - 2) flops, i.e. 28 at k = 1 (Sec. III).
The minimum HBM traffic of a pass is one read and one write of the state,
16 bytes per amplitude, so the read+write arithmetic intensity is
(8 * 2^k - 2) / 16 flop/B.
"""

AMP_BYTES = 8  # complex64


def flops_per_group(k: int) -> int:
    return (1 << k) * (8 * (1 << k) - 2)


def useful_flops(n: int, k: int) -> int:
    return (1 << (n - k)) * flops_per_group(k)


def bytes_per_pass(n: int) -> int:
    return 2 * AMP_BYTES * (1 << n)


def ai_read_write(k: int) -> float:
    return (8 * (1 << k) - 2) / 16.0
