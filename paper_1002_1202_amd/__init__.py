"""Generalized shifted COCG for non-orthogonal tight-binding pairs on MI355X.

The compute path is the HIP library ``libgsc.so`` (C ABI in include/gsc.h);
``paper_1002_1202_amd.api`` only marshals arguments to it.  Importing the
package does not load the library; the first call does, and fails loudly if
it is missing.
"""
from ._lib import GscError, load  # noqa: F401
