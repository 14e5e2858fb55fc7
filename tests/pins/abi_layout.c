/* Prints the sizes and a few offsets of the C ABI structs (compiled by the tests). */
#include <stddef.h>
#include <stdio.h>

#include "fpt.h"

int main(void) {
    printf("fpt_spectrum %zu\n", sizeof(fpt_spectrum));
    printf("fpt_dye %zu\n", sizeof(fpt_dye));
    printf("fpt_medium %zu\n", sizeof(fpt_medium));
    printf("fpt_sphere %zu\n", sizeof(fpt_sphere));
    printf("fpt_scene_desc %zu\n", sizeof(fpt_scene_desc));
    printf("fpt_run %zu\n", sizeof(fpt_run));
    printf("fpt_tune %zu\n", sizeof(fpt_tune));
    printf("fpt_path_record %zu\n", sizeof(fpt_path_record));
    printf("off_geometry %zu\n", offsetof(fpt_scene_desc, geometry));
    printf("off_light %zu\n", offsetof(fpt_scene_desc, light));
    printf("off_sensor %zu\n", offsetof(fpt_scene_desc, sensor));
    printf("off_fov %zu\n", offsetof(fpt_scene_desc, fov_y_deg));
    printf("off_gloss %zu\n", offsetof(fpt_scene_desc, wall_gloss));
    printf("off_splat_rr %zu\n", offsetof(fpt_run, splat_rr));
    return 0;
}
