"""MI355X-native transpose of row-distributed XCSR multigraphs (arXiv 2012.06012).

The compute path is libmgt.so (hand-written HIP for gfx950) behind a C ABI;
``paper_2012_06012_amd.mgt`` is its thin Python binding. Importing the binding
fails loudly if the library has not been built.
"""
__all__ = ["mgt"]
