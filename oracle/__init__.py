"""Plain, slow, FP64 CPU oracle of randomized HODLR / HBS compression.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) may import, call, link or execute anything in this package.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.

It follows Martinsson, "Compressing rank-structured matrices via randomized
sampling" (arXiv 1503.07152) step by step, in the paper's order and notation,
with NumPy/LAPACK primitives (matmul, QR, SVD) as its only library steps:

* ``tree``     -- the binary index tree (Sec. 2.7, Fig. 1).
* ``rng``      -- Gaussian test matrices (``randn`` of Fig. 2/4) from a
                 counter-based Philox4x32-10 stream with Box-Muller.
* ``lowrank``  -- ``qr``/``svd``/``id`` in their three modes (Sec. 2.2-2.4, 2.6).
* ``hbs``      -- HBS representation, the partial apply of Fig. 7, the
                 storage-efficient compression of Fig. 4 and the HBS-ID
                 post-sweep of Fig. 5.
* ``hodlr``    -- HODLR representation and the compression of Fig. 2.
* ``operators``-- black-box operators: dense and kernel matrices, synthetic
                 HBS applied in O(N k).
* ``metrics``  -- the randomized error estimate E of Sec. 5 and exact errors.
* ``grad``     -- reference gradients of the compressed apply (plain dense
                 assembly differentiated by torch CPU autograd).

It shares no code with the HIP path.
"""
