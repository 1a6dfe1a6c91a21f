"""MI355X-native D3Q19 LBM-LES hot path (arXiv 2607.04516, App. D).

The compute lives in liblbm.so (HIP, gfx950) behind the C ABI of
include/lbm.h; ``binding`` marshals arguments to it, ``workloads`` builds the
seeded synthetic inputs.
"""
