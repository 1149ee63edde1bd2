"""MI355X-native HARM ideal-GRMHD step: HIP kernels behind a C ABI.

`paper_2408_01361_amd.grmhd` binds libgrmhd.so (built by
`paper_2408_01361_amd.build.build()`); import it explicitly so that a missing
library fails loudly at that import.
"""
