"""MI355X (gfx950) fast edge-aware occlusion detection.

The detector (Sippel, Seiler, Kaup, ICIP 2024, Sec. 3) runs in the HIP
kernels of ``libocclusion.so`` behind the C ABI of ``include/occl.h``;
``paper_2408_14050_amd.occl`` is its ctypes binding and
``paper_2408_14050_amd.scenes`` the seeded synthetic input generator.
"""
__all__ = ["occl", "scenes"]
