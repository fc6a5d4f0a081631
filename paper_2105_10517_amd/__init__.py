"""MI355X-native split-step Crank-Nicolson solver for the rotating spin-1
spin-orbit- and Rabi-coupled Gross-Pitaevskii equation (arXiv:2105.10517).

Importing the package is cheap: the HIP library is loaded on first use by
``paper_2105_10517_amd.binding`` and raises if it has not been built.
"""
__all__ = ["inputs"]
