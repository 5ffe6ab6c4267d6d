"""MI355X implicit cloth step (P-Cloth hot path): HIP kernels behind a C ABI.

``binding`` loads ``libpcloth.so`` (built by ``build.py``); ``meshgen`` makes
the seeded synthetic inputs.
"""
__all__ = ["binding", "meshgen"]
