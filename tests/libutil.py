"""Helpers shared by the tests: build libqpe.so only if it is not built yet."""
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2507_17175_amd", "libqpe.so")


def ensure_built() -> str:
    if not os.path.exists(LIB):
        from paper_2507_17175_amd.build import build
        build()
    return LIB
