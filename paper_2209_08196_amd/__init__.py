"""MI355X-native Jiffy LiDAR scan codec.

The codec runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/jiffy.h`` (``libjiffy.so``); ``paper_2209_08196_amd.jiffy`` is the
thin Python binding over it, with PyTorch used for device memory and streams.
``paper_2209_08196_amd.synth`` generates seeded synthetic scan sequences.
"""
