"""MI355X (gfx950) implementation of the sparse stress model's hot path.

``graphs`` holds the seeded input generators; ``ssm`` is the thin ctypes
binding of the HIP library ``libssm.so`` (loaded on first use)."""
__all__ = ["graphs", "ssm"]
