"""Exact subgraph counting on MI355X: pattern-aware DFS subgraph extension
(arXiv 2112.09761) as a C-ABI HIP library (libgpm.so) with a thin Python
binding (``paper_2112_09761_amd.gpm``) and seeded input generators
(``paper_2112_09761_amd.synth``).

Importing the package loads nothing native; ``gpm.lib()`` loads libgpm.so and
raises if it has not been built.
"""
