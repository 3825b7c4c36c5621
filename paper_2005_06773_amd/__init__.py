"""MI355X-native multi-hypothesis criticality (Sanchez Morales et al., IEEE IV 2019).

``paper_2005_06773_amd.mhc``      ctypes binding of libmhc.so (C ABI in include/mhc.h)
``paper_2005_06773_amd.scenegen`` seeded synthetic scenes (inputs only)
``paper_2005_06773_amd.build``    hipcc build of libmhc.so for gfx950
"""
__all__ = ["mhc", "scenegen", "build"]
