"""MI355X (gfx950) hash-based sector carving: a C-ABI HIP library and its binding.

The library (`libcarve.so`, built from `csrc/`) exports build_master_index,
scan_image, flagged_sectors and confirm_matches (see include/carve.h). The
binding lives in `carve.py`; importing this package loads nothing.
"""

__all__ = ["carve"]
