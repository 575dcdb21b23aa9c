"""Benchmark placeholder (filled in with the device path)."""


def cell_updates_per_s(n: int, seconds: float) -> float:
    """Throughput of one APSP solve: n^3 cell updates over the wall time (Sec. 5.4)."""
    return float(n) ** 3 / seconds
