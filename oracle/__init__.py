"""CPU oracle for the two-site shell-model DMRG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library and
its Python binding) imports, links or executes anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.

* `ed`      - exact diagonalisation in the m-scheme basis (Eq. 1 applied to
              Slater determinants), the plain definition of the ground state.
* `dmrg`    - a plain FP64 NumPy two-site DMRG (superblock of two blocks and two
              explicit sites, density-matrix truncation, back-and-forth sweeps),
              written from the method description, merged-sector dense blocks.
* `hashrand`- SplitMix64 keyed hashing for the method's random start.
* `entropy` - one- and two-orbital entropies, mutual information and the
              Fiedler-vector ordering, from their definitions.
"""
