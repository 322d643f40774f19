"""Seeded synthetic inputs shared by the oracle-side and HIP-side tests.

Holds no solver arithmetic (see phantoms' header)."""
from .phantoms import *  # noqa: F401,F403
