"""MI355X-native layered normalised min-sum LDPC decoder (gfx950 HIP kernels
behind the C ABI of include/ldpc.h). Import ``paper_2009_05534_amd.ldpc``
for the binding; importing this package loads nothing."""
__version__ = "0.1.0"
