"""fibersim: per-cycle bulk-synchronous RTL simulation of fiber-partitioned
netlists on MI355X (gfx950).

Importing the package loads nothing native.  ``paper_2403_04714_amd.fibersim``
is the binding of the C-ABI library ``libfibersim.so``; ``netgen`` builds
seeded synthetic netlists.
"""
