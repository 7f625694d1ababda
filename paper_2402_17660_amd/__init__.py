"""MI355X TensorNet energy-and-forces library (Python binding of libtensornet.so)."""

from .api import Graph, TensorNet, TensorNetEF, TensorNetError, Workspace, build_neighbors, capture  # noqa: F401
from ._lib import LIB_PATH, LibraryMissing, lib  # noqa: F401
