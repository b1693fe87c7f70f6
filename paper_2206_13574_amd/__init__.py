"""Graph wavefront alignment (Gwfa) on AMD MI355X (gfx950).

The HIP library is loaded on first use by :mod:`paper_2206_13574_amd.gwfa`;
importing the package itself loads nothing.
"""
