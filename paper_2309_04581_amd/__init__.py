"""MI355X-native hybrid surface-volumetric marcher (radiance field + meshes).

The rendering path lives in the HIP library ``libmeshrf.so`` behind a C ABI
(``include/meshrf.h``); :mod:`paper_2309_04581_amd.meshrf` is its thin ctypes
binding.  :mod:`paper_2309_04581_amd.scenegen` draws the seeded synthetic inputs.
"""
