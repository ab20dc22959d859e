"""Exact multidimensional range queries on MI355X (gfx950).

The GPU library (``lib/libmdrq.so``) is loaded lazily by :mod:`.mdrq`; importing
the package itself loads nothing.
"""
