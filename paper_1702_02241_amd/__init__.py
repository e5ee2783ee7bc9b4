"""Split-SPCP (Burer-Monteiro robust PCA, sparse part marginalised) on MI355X.

* ``rpca``   -- ctypes binding of the C ABI in ``include/rpca.h`` (librpca.so)
* ``torch_api`` -- convenience wrappers taking torch device tensors
* ``synth``  -- seeded synthetic workloads (data only, no method arithmetic)
* ``build``  -- compiles librpca.so for gfx950 in-tree
"""
