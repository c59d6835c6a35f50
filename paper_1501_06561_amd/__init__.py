"""Frequent Directions family of row-streaming matrix sketches on MI355X (gfx950).

The compute path is the HIP library ``libfdsketch.so`` built from ``csrc/``;
``fdsketch`` is its thin ctypes binding.  ``synth`` draws seeded inputs.
Importing the package does not load the library; ``fdsketch.lib()`` does.
"""
__all__ = ["synth", "fdsketch"]
