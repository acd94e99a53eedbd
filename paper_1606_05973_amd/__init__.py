"""gfx950 (MI355X) two-pass connected component labeling after Gupta et al.,
arXiv 1606.05973.

    from paper_1606_05973_amd import ccl      # loads libccl.so (raises if unbuilt)
    labels = ccl.label(img_u8_cuda, conn=8)

Submodules: ``ccl`` (binding of include/ccl.h), ``build`` (hipcc build of
libccl.so), ``inputs`` (seeded synthetic images), ``autotune`` (tile choice),
``serve`` (continuous-batching request loop).
"""
