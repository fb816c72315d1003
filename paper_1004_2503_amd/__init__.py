"""MI355X-native explicit M1 radiative transfer with hydrogen photo-chemistry
(the per-step hot path of Aubert & Teyssier 2010, "Reionization simulations
powered by GPUs I").

The compute path is the C-ABI library ``librt_m1.so`` (hand-written HIP for
gfx950); ``paper_1004_2503_amd.rt`` is its thin ctypes binding and
``paper_1004_2503_amd.workloads`` the seeded synthetic inputs.  Importing the
package loads nothing; the binding loads the library on first use and raises
if it has not been built.
"""

__version__ = "0.1.0"
