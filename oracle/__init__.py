"""CPU oracle of the pruned, per-shape-selected GEMM method.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs
anything here; only ``tests/``, the smoke entry point and the benchmark's
CPU-baseline leg do.  The oracle shares no code with the library: its inputs
come from the ``synth`` module (seeded generators, no arithmetic of the method).

Each module follows one passage of the paper (J. Lawson, "Performance
portability through machine learning guided kernel selection in SYCL
libraries", arXiv 2008.13145) and says which:

* ``gemm``       -- section 3: the matrix multiply itself (FP64 triple loop in C).
* ``normalize``  -- section 3.4: relative, raw-cutoff, standard-cutoff and
                    sigmoid normalization of one problem's performance vector.
* ``kmeans``     -- section 4.1 (k-means) and 4.2 (centroid -> kernel, Top-N).
* ``pca``        -- section 4.1 (PCA before k-means) and the pruning built on it.
* ``represent``  -- section 4.2: a cluster's kernel from a representative or
                    from the geometric mean of its members.
* ``prune_tree`` -- section 4.1: decision-tree pruning to k leaves.
* ``conv``       -- section 6: direct convolution and pooling (VGG16 layers).
* ``cart``       -- section 5.1: decision-tree classifiers A/B/C.
* ``regret``     -- section 4.3: fraction of optimal performance, geometric mean.
* ``mlp``        -- the MLP cost model that stands in for the decision tree
                    (section 5.1 lists an MLP among the classifiers); FP64.
* ``convert``    -- BF16 and FP8-e4m3 rounding used by the low-precision paths.

Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
brute force, invariants or library routines.  No function is parity unpinned.
"""
