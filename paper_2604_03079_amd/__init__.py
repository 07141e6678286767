"""Coloured, conflict-free MOSFET evaluate-and-stamp for MI355X (gfx950).

The GPU library is loaded lazily by ``paper_2604_03079_amd.colorstamp``; importing
the package itself does not touch the GPU."""
