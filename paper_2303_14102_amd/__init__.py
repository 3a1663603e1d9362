"""MI355X (gfx950) linear-complexity Silhouette (arXiv 2303.14102): squared Euclidean and cosine.

The computation lives in the HIP library libsilhouette.so behind the C ABI of
include/silhouette.h; ``silhouette`` and ``cluster_stats`` are thin torch-facing bindings.
"""

from .binding import (BatchedSilhouette, SilhouetteFn, cluster_stats, kmeans_step,  # noqa: F401
                      silhouette, silhouette_backward, silhouette_mahalanobis, silhouette_stream, status,
                      stream_workspace_bytes, workspace_bytes)
