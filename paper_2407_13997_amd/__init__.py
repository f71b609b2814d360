"""Space-time waveform-relaxation multigrid for Navier-Stokes on MI355X.

The compute path is the gfx950 library ``libstwr.so`` (C ABI in
``include/stwr.h``); this package only marshals arguments to it.  Import the
binding with ``from paper_2407_13997_amd import binding``.
"""
__all__ = ["binding", "build"]
