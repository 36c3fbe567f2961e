"""MI355X-native RAPID coarse-to-fine superpixel refinement sweep."""
